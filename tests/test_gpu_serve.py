"""Serving: every request's rows alone == inside a mix, bit for bit.

A server over three resident tables takes a mix of uniform, shape-restricted
and classified sample requests of many sizes plus AGS rounds from one session
per table. Each sample request must equal scc_sample / scc_classify called on
its own with the same (table, shape, seed, stream, first index), and one is
also checked against the oracle; each AGS session must pick the shapes and
reach the counts of scc_ags with the same round size (and of the oracle's AGS).
The first-in first-out mode, age-weighted shares and small-first steps must give the same rows. Admission: a request that
does not fit the budget waits until earlier outputs are released; a request
larger than the budget is refused with ENOMEM, and a full queue with EBUSY.
"""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from gpu_util import scc

pytestmark = pytest.mark.gpu


def _tables():
    S = scc()
    specs = [(gg.chung_lu(3000, 12000, 2.2, 150, seed=41), 5),
             (gg.barabasi_albert(1500, 3, seed=42), 6),
             (gg.erdos_renyi(2000, 8000, seed=43), 4)]
    out = []
    for i, (g, k) in enumerate(specs):
        colors = gg.colors(g.n, k, seed=50 + i)
        out.append((g, colors, k, S.Table(S.DeviceGraph.from_graph(g), colors, k)))
    return out


def _requests(tabs, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        t = i % len(tabs)
        tab = tabs[t][3]
        n = int(np.exp(rng.uniform(np.log(5), np.log(20000))))
        tj = tab.totals()[1]
        shapes = [j for j, x in enumerate(tj) if x > 0]
        shape = -1 if rng.random() < 0.6 else int(rng.choice(shapes))
        reqs.append(dict(table=t, n=n, seed=int(rng.integers(1, 1 << 40)), stream_id=int(rng.integers(0, 100)),
                         first_index=int(rng.integers(0, 1 << 30)), shape=shape, classify=bool(rng.random() < 0.5)))
    return reqs


def _alone(tab, q):
    import torch
    v, p = tab.sample(q["n"], seed=q["seed"], stream_id=q["stream_id"], shape=q["shape"],
                      first_index=q["first_index"])
    cls = None
    if q["classify"]:
        _, cls = tab.classify(v)
        cls = cls.cpu().numpy()
    torch.cuda.synchronize()
    return v.cpu().numpy(), p.cpu().numpy(), cls


def _run(srv, reqs, sessions, rounds, round_size):
    """Submits the sample requests with the AGS rounds interleaved; returns results by position."""
    ids = []
    order = []
    ags_ids = []
    per = max(1, len(reqs) // max(1, rounds))
    for i, q in enumerate(reqs):
        ids.append(srv.submit(**q))
        order.append(i)
        if i % per == 0:
            for t, sid in enumerate(sessions):
                if sum(1 for x in ags_ids if x[0] == t) < rounds:
                    ags_ids.append((t, srv.submit(t, round_size, session=sid)))
    for t, sid in enumerate(sessions):
        while sum(1 for x in ags_ids if x[0] == t) < rounds:
            ags_ids.append((t, srv.submit(t, round_size, session=sid)))
    out = []
    for rid in ids:
        r = srv.wait(rid)
        assert r["status"] == 0
        out.append(r)
        srv.release(rid)
    for _, rid in ags_ids:
        r = srv.wait(rid)
        assert r["status"] == 0
        srv.release(rid)
    return out


def test_mix_equals_alone_and_ags_equals_plain():
    S = scc()
    tabs = _tables()
    reqs = _requests(tabs, 45, seed=7)
    srv = S.Server([t[3] for t in tabs], hbm_budget=48 << 20, step_samples=4096, chunk=256)
    sessions = [srv.ags_open(t, cbar=15, seed=300 + t, stream_id=t) for t in range(len(tabs))]
    rounds, rsize = 4, 700
    res = _run(srv, reqs, sessions, rounds, rsize)
    st = srv.stats()
    assert st["completed"] == len(reqs) + rounds * len(tabs)
    assert st["samples"] == sum(q["n"] for q in reqs) + rounds * rsize * len(tabs)
    assert st["arena_used"] == 0 and st["p50_ms"] <= st["p99_ms"]
    for q, r in zip(reqs, res):
        v, p, cls = _alone(tabs[q["table"]][3], q)
        assert r["shape"] == q["shape"] and r["first_index"] == q["first_index"]
        assert np.array_equal(r["verts"].cpu().numpy(), v), q
        assert np.array_equal(r["parent"].cpu().numpy(), p), q
        if q["classify"]:
            assert np.array_equal(r["cls"].cpu().numpy(), cls), q
        else:
            assert r["cls"] is None
    # one request against the oracle directly
    q = next(x for x in reqs if x["table"] == 0 and x["n"] <= 2000)
    g, colors, k, _ = tabs[0]
    ov, op = O.Table(g, colors, k).sample(q["n"], seed=q["seed"], stream=q["stream_id"], shape=q["shape"],
                                          first_index=q["first_index"])
    r = res[reqs.index(q)]
    assert np.array_equal(r["verts"].cpu().numpy(), ov) and np.array_equal(r["parent"].cpu().numpy(), op)
    # AGS sessions: the rounds of scc_ags with the same round size
    for t, sid in enumerate(sessions):
        got = srv.ags_result(sid, t)
        ref = tabs[t][3].ags(cbar=15, round_size=rsize, budget=rounds * rsize, seed=300 + t, stream_id=t)
        assert len(ref["round_shapes"]) == rounds   # no session covers every class this early
        for key in ("hits", "w", "n_j", "round_shapes"):
            assert np.array_equal(got[key], ref[key]), (t, key)
    g, colors, k, _ = tabs[1]
    oref = O.Table(g, colors, k).ags(cbar=15, round_size=rsize, budget=rounds * rsize, seed=301, stream=1)
    got = srv.ags_result(sessions[1], 1)
    for key in ("hits", "w", "n_j", "round_shapes"):
        assert np.array_equal(got[key], oref[key]), key
    srv.close()


def test_fifo_mode_gives_the_same_rows():
    S = scc()
    tabs = _tables()
    reqs = _requests(tabs, 12, seed=11)
    mix = S.Server([t[3] for t in tabs], hbm_budget=32 << 20, step_samples=2048, chunk=128)
    fifo = S.Server([t[3] for t in tabs], hbm_budget=32 << 20, fifo=True)
    aged = S.Server([t[3] for t in tabs], hbm_budget=32 << 20, step_samples=2048, chunk=128, age_tau=0.002)
    small = S.Server([t[3] for t in tabs], hbm_budget=32 << 20, step_samples=2048, small_request=600,
                     small_step=512)
    a = _run(mix, reqs, [], 0, 1)
    b = _run(fifo, reqs, [], 0, 1)
    c = _run(aged, reqs, [], 0, 1)
    d = _run(small, reqs, [], 0, 1)
    for ra, rb, rc, rd in zip(a, b, c, d):
        assert np.array_equal(ra["verts"].cpu().numpy(), rb["verts"].cpu().numpy())
        assert np.array_equal(ra["parent"].cpu().numpy(), rb["parent"].cpu().numpy())
        assert np.array_equal(ra["verts"].cpu().numpy(), rc["verts"].cpu().numpy())
        assert np.array_equal(ra["verts"].cpu().numpy(), rd["verts"].cpu().numpy())
        assert np.array_equal(ra["parent"].cpu().numpy(), rd["parent"].cpu().numpy())
    assert fifo.stats()["steps"] >= len(reqs)
    for srv in (mix, fifo, aged, small):
        srv.close()


def test_small_first_mode_with_ags_rounds():
    # small requests first, then submission order, steps cut while a small one
    # runs: rows and AGS sessions as with shares
    S = scc()
    tabs = _tables()
    reqs = _requests(tabs, 30, seed=13)
    srv = S.Server([t[3] for t in tabs], hbm_budget=48 << 20, step_samples=4096, small_request=1000, small_step=1024)
    sessions = [srv.ags_open(t, cbar=15, seed=300 + t, stream_id=t) for t in range(len(tabs))]
    rounds, rsize = 3, 700
    res = _run(srv, reqs, sessions, rounds, rsize)
    for q, r in zip(reqs, res):
        v, p, cls = _alone(tabs[q["table"]][3], q)
        assert np.array_equal(r["verts"].cpu().numpy(), v) and np.array_equal(r["parent"].cpu().numpy(), p), q
        if q["classify"]:
            assert np.array_equal(r["cls"].cpu().numpy(), cls), q
    for t, sid in enumerate(sessions):
        got = srv.ags_result(sid, t)
        ref = tabs[t][3].ags(cbar=15, round_size=rsize, budget=rounds * rsize, seed=300 + t, stream_id=t)
        for key in ("hits", "w", "n_j", "round_shapes"):
            assert np.array_equal(got[key], ref[key]), (t, key)
    srv.close()


def test_admission_by_budget():
    S = scc()
    tabs = _tables()
    tab = tabs[0][3]   # k = 5
    n = 4096
    need = ((n * 5 * 4 + 255) // 256 + (n * 4 + 255) // 256 + (n * 5 + 255) // 256) * 256
    srv = S.Server([tab], hbm_budget=int(need * 1.5), max_pending=2)
    # larger than the whole budget: refused
    with pytest.raises(S.SccError) as e:
        srv.submit(0, 3 * n, seed=1)
    assert e.value.status == S.ENOMEM
    a = srv.submit(0, n, seed=1)
    ra = srv.wait(a)                       # a holds its outputs until released
    b = srv.submit(0, n, seed=2)
    c = srv.submit(0, n, seed=3)
    with pytest.raises(S.SccError) as e:   # two requests already wait for admission
        srv.submit(0, n, seed=4)
    assert e.value.status == S.EBUSY
    with pytest.raises(S.SccError) as e:   # b cannot start while a holds the budget
        srv.wait(b, timeout=0.3)
    assert e.value.status == S.EBUSY
    srv.release(a)
    rb = srv.wait(b)
    assert rb["t_admit"] >= ra["t_done"]
    srv.release(b)
    rc = srv.wait(c)
    assert rc["t_admit"] >= rb["t_done"]
    v, p, _ = _alone(tab, dict(n=n, seed=3, stream_id=0, shape=-1, first_index=0, classify=False))
    assert np.array_equal(rc["verts"].cpu().numpy(), v)
    srv.release(c)
    st = srv.stats()
    assert st["rejected"] == 1 and st["completed"] == 3 and st["arena_used"] == 0
    srv.close()
