"""The allocation-free sampling entry point (scc_sample_noalloc) against scc_sample.

Both are called through the C ABI on the same table and arguments: uniform and
shape-restricted streams on a graph with hub rows (their running sums come
with the build), two calls in a row with the second smaller (the shared
scratch keeps the last call's flags and must be cleared), and the refusal to
draw from running sums that are not built yet.
"""
from __future__ import annotations

import pytest
import torch

import graphgen as gg
from gpu_util import scc

pytestmark = pytest.mark.gpu


def _table(k=6):
    S = scc()
    g = gg.chung_lu(6000, 30000, 2.1, 1500, seed=61)
    colors = gg.colors(g.n, k, seed=62)
    return S, S.Table(S.DeviceGraph.from_graph(g), colors, k, hub_degree=256)


def _pair(tab, n, seed, shape=-1, first=0):
    ref_v, ref_p = tab.sample(n, seed=seed, shape=shape, first_index=first)
    v = torch.full((n, tab.k), -7, dtype=torch.int32, device="cuda")
    p = torch.full((n, tab.k), 9, dtype=torch.int8, device="cuda")
    tab.sample_noalloc(v, p, seed=seed, shape=shape, first_index=first)
    torch.cuda.synchronize()
    return ref_v, ref_p, v, p


def test_noalloc_equals_sample_twice_second_smaller():
    S, tab = _table()
    assert tab.info().num_hubs > 0
    for n, seed, first in [(5000, 3, 0), (777, 4, 123)]:
        print("noalloc uniform", n, seed, first, flush=True)
        rv, rp, v, p = _pair(tab, n, seed, first=first)
        assert torch.equal(rv, v) and torch.equal(rp, p), n


def test_noalloc_shapes_after_preparation():
    S, tab = _table()
    nu = tab.info().num_unrooted
    t, tj = tab.totals()
    for j in range(nu):
        if tj[j] == 0:
            continue
        v = torch.empty((10, tab.k), dtype=torch.int32, device="cuda")
        p = torch.empty((10, tab.k), dtype=torch.int8, device="cuda")
        with pytest.raises(S.SccError) as e:       # shape j's running sums do not exist yet
            tab.sample_noalloc(v, p, seed=1, shape=j)
        assert e.value.status == S.EINVAL
        for n in (3000, 100):
            print("noalloc shape", j, n, flush=True)
            rv, rp, v, p = _pair(tab, n, seed=5 + j, shape=j)
            assert torch.equal(rv, v) and torch.equal(rp, p), (j, n)


def test_noalloc_arguments():
    S, tab = _table(5)
    v = torch.empty((4, 5), dtype=torch.int32, device="cuda")
    p = torch.empty((4, 5), dtype=torch.int8, device="cuda")
    with pytest.raises(S.SccError) as e:
        tab.sample_noalloc(v, p, seed=1, shape=99)
    assert e.value.status == S.EINVAL
    tab.sample_noalloc(v[:0], p[:0], seed=1)       # n = 0: nothing to do


def test_noalloc_before_any_sample():
    """Before the first scc_sample the table has no per-edge colour copy, and the
    neighbour draw reads the colour array instead: the samples are the same."""
    S, tab = _table()
    n = 3000
    v = torch.full((n, tab.k), -7, dtype=torch.int32, device="cuda")
    p = torch.full((n, tab.k), 9, dtype=torch.int8, device="cuda")
    print("noalloc before any sample", n, flush=True)
    tab.sample_noalloc(v, p, seed=9, first_index=11)
    torch.cuda.synchronize()
    rv, rp = tab.sample(n, seed=9, first_index=11)
    assert torch.equal(rv, v) and torch.equal(rp, p)
    print("noalloc after the first sample", n, flush=True)
    rv2, rp2, v2, p2 = _pair(tab, n, seed=9, first=11)
    assert torch.equal(rv2, v) and torch.equal(v2, v) and torch.equal(p2, p)
