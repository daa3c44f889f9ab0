"""Variable-length counts (Sec. 3.3) on the GPU: a table re-encoded after the
build answers every query exactly as the fixed-layout table and the oracle.

* Every level (offsets, keys, both count words), t and t_j equal the oracle's
  on random graphs for every k in [2, 8] under zero-rooting, all rootings and
  round skipping; counts up to 16 bytes (the 2^16-leaf star at k = 6, about
  1e22 copies, and the 2^17-leaf hub at k = 7).
* Sample streams (uniform, every shape, stars under round skipping), occ
  queries, AGS runs and served requests equal the fixed-layout table's.
* The full mid-size workload (Chung-Lu n = 1e6, m = 1e7, k = 6): every level of
  the re-encoded table equals the fixed-layout one (itself pinned to the oracle
  at that size) and the records take less than 70 % of the bytes.
"""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from gpu_util import assert_tables_equal, random_graphs, scc

pytestmark = pytest.mark.gpu


def _pair(g, colors, k, rooting=O.ROOT_ZERO):
    S = scc()
    dg = S.DeviceGraph.from_graph(g)
    return S.Table(dg, colors, k, rooting=rooting, vlc=True), S.Table(dg, colors, k, rooting=rooting)


def _same_samples(a, b, n, seed, shape=-1, stream=0):
    av, ap = a.sample(n, seed=seed, stream_id=stream, shape=shape)
    bv, bp = b.sample(n, seed=seed, stream_id=stream, shape=shape)
    return np.array_equal(av.cpu().numpy(), bv.cpu().numpy()) and np.array_equal(ap.cpu().numpy(), bp.cpu().numpy())


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("rooting", [O.ROOT_ZERO, O.ROOT_ALL, O.ROOT_BALANCED])
def test_vlc_tables_every_k(k, rooting):
    if rooting == O.ROOT_BALANCED and k < 4:
        pytest.skip("round skipping needs k >= 4")
    for name, g in random_graphs(k):
        colors = gg.colors(g.n, k, seed=29 * k + rooting)
        vt, ft = _pair(g, colors, k, rooting)
        ot = O.Table(g, colors, k, rooting)
        assert vt.info().vlc == 1
        assert_tables_equal(vt, ot, k, f"{name} vlc")
        t, tj = ot.totals()
        if t:
            assert _same_samples(vt, ft, 400, seed=k, stream=3), name
        for j in range(O.num_unrooted(k)):
            w = ot.star_count() if rooting == O.ROOT_BALANCED and j == O.star_class(k) else tj[j]
            if w:
                assert _same_samples(vt, ft, 100, seed=j + 1, shape=j, stream=j), (name, j)
        rng = np.random.default_rng(k)
        for _ in range(20):
            v = int(rng.integers(g.n))
            key = int(rng.integers(-1, O.num_keys(k)))
            assert vt.occ(v, key) == ft.occ(v, key)


@pytest.mark.parametrize("k,leaves,ncol", [(6, 1 << 16, 5), (7, 1 << 17, 6)])
def test_vlc_wide_counts(k, leaves, ncol):
    edges = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 1) for i in range(1, 200)]
    g = gg.csr_from_edges(leaves + 1, np.array(edges, np.int64))
    colors = np.concatenate([[0], (np.arange(leaves) % ncol) + 1]).astype(np.uint8)
    vt, ft = _pair(g, colors, k)
    assert_tables_equal(vt, O.Table(g, colors, k, O.ROOT_ZERO), k, "wide vlc")
    assert vt.totals()[0] > 2 ** 64
    assert _same_samples(vt, ft, 3000, seed=5)
    assert vt.occ(0, -1) == ft.occ(0, -1) > 2 ** 64


def test_vlc_ags_and_server():
    S = scc()
    g = gg.chung_lu(3000, 12000, 2.2, 150, seed=71)
    k = 6
    colors = gg.colors(g.n, k, seed=72)
    vt, ft = _pair(g, colors, k)
    a = vt.ags(cbar=20, round_size=500, budget=6000, seed=9)
    b = ft.ags(cbar=20, round_size=500, budget=6000, seed=9)
    for key in ("hits", "w", "n_j", "round_shapes"):
        assert np.array_equal(a[key], b[key]), key
    srv = S.Server([vt, ft], hbm_budget=16 << 20, step_samples=2048, chunk=128)
    ids = [srv.submit(t, 3000, seed=11 + i, shape=-1, classify=True) for i, t in enumerate([0, 1, 0, 1])]
    rows = [srv.wait(r) for r in ids]
    assert np.array_equal(rows[0]["verts"].cpu().numpy(), ft.sample(3000, seed=11)[0].cpu().numpy())
    assert np.array_equal(rows[2]["verts"].cpu().numpy(), ft.sample(3000, seed=13)[0].cpu().numpy())
    for r in ids:
        srv.release(r)
    srv.close()


@pytest.mark.timeout(600)
def test_vlc_mid_workload_full_table():
    k = 6
    g = gg.chung_lu(1_000_000, 10_000_000, 2.1, 5e4, seed=2)
    colors = gg.colors(g.n, k, seed=12)
    vt, ft = _pair(g, colors, k)
    vi, fi = vt.info(), ft.info()
    print(f"mid: records {vi.record_bytes / 1e9:.3f} GB vs {fi.record_bytes / 1e9:.3f} GB, table "
          f"{vi.bytes / 1e9:.2f} GB vs {fi.bytes / 1e9:.2f} GB", flush=True)
    assert vi.record_bytes < 0.7 * fi.record_bytes
    for h in range(1, k + 1):
        for a, b in zip(vt.export_level(h), ft.export_level(h)):
            assert np.array_equal(a, b), h
    assert vt.totals() == ft.totals()
    assert _same_samples(vt, ft, 100_000, seed=22)
