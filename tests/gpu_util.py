"""Helpers shared by the GPU parity tests: build both sides on the same seeded input."""
from __future__ import annotations

import numpy as np

import graphgen as gg
import oracle as O


def scc():
    import paper_2009_03052_amd as S
    return S


def build_pair(g, colors, k, rooting=0, validate=True, hub_degree=0, gather_mode=0, width_test=0):
    S = scc()
    dg = S.DeviceGraph.from_graph(g)
    gt = S.Table(dg, colors, k, rooting=rooting, validate=validate, hub_degree=hub_degree, gather_mode=gather_mode,
                 width_test=width_test)
    ot = O.Table(g, colors, k, rooting)
    return gt, ot


def assert_tables_equal(gt, ot, k, label=""):
    for h in range(1, k + 1):
        go, gk, gl, gh = gt.export_level(h)
        oo, ok_, ol, oh = ot.export_level(h)
        assert np.array_equal(go, oo), f"{label} level {h}: offsets differ"
        assert np.array_equal(gk, ok_), f"{label} level {h}: keys differ"
        assert np.array_equal(gl, ol), f"{label} level {h}: low words differ"
        assert np.array_equal(gh, oh), f"{label} level {h}: high words differ"
    assert gt.totals() == ot.totals(), f"{label}: totals differ"


def assert_samples_equal(gt, ot, n, seed, stream=0, shape=-1, first=0, label=""):
    gv, gp = gt.sample(n, seed=seed, stream_id=stream, shape=shape, first_index=first)
    ov, op = ot.sample(n, seed=seed, stream=stream, shape=shape, first_index=first)
    gv = gv.cpu().numpy()
    gp = gp.cpu().numpy()
    assert np.array_equal(gv, ov), f"{label}: sample vertices differ"
    assert np.array_equal(gp, op), f"{label}: sample parents differ"
    return gv


def random_graphs(k):
    """(name, graph) cases for one k: ER, Chung-Lu, BA and a few structured graphs."""
    out = []
    n_er = 70 if k <= 6 else 45
    out.append((f"er-k{k}", gg.erdos_renyi(n_er, 3 * n_er, seed=200 + k)))
    out.append((f"cl-k{k}", gg.chung_lu(300, 900, 2.2, 40, seed=300 + k)))
    out.append((f"ba-k{k}", gg.barabasi_albert(120, 2, seed=400 + k)))
    out.append((f"lollipop-k{k}", gg.lollipop(9, 4)))
    return out
