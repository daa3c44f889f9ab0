"""Benchmark: the whole hot path on one MI355X.

Default workload (large): one step = table build (Eq. (1) DP, all levels,
totals) + 10^7 uniform colourful 8-treelet samples + their classification, on a
Chung-Lu graph with n = 4*10^6, m = 6*10^7, exponent 2.3, maximum expected
degree 2*10^5 (seeded), k = 8, zero-rooting, counts 64- or 128-bit by the
per-vertex bound. The graph and colours are resident in HBM before timing
starts. `--workload mid` runs the same step at k = 6 on the mid graph;
`batching` and `serving` run the project's batched build and request server.

Prints one JSON line. `value` is classified samples per second of whole steps
(build included). The roofline entry is the DP join (neighbour-sum gather,
combine with compaction and packing, level-k totals): the algorithmic bytes of
its launches divided by their duration, measured with HIP events on the
build's stream; `roofline_parts` splits it into the gather and the combine and
adds the sampler. The large line also carries `batched_vs_plain` and
`served_vs_fifo`: the batching workload with three timed steps per group, and
the serving workload's trace through continuous batching and first-in first-out
only (`--no-companions` leaves them out).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--samples", type=int, default=None, help="samples per step (default: the workload's)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-round-skipping", action="store_true",
                   help="leave out the extra round-skipping, biased-colouring and variable-length builds "
                        "(counter runs: only the plain step's kernels)")
    p.add_argument("--small", action="store_true", help="small graph (for quick checks)")
    p.add_argument("--workload", default="large", choices=["mid", "large", "batching", "serving", "k16"],
                   help="large (default) / mid: the plain method on the large / mid graph; batching: 48 "
                        "instances, plain vs one "
                        "batched launch; serving: three resident k=7 tables under a Poisson request mix, continuous "
                        "batching vs first-in first-out; k16: the sparse-record build for k up to 16 "
                        "(k = 10 on a sparse Chung-Lu graph)")
    p.add_argument("--serve-step", type=int, default=1 << 18,
                   help="serving: samples per step of the continuous-batching server (its share granularity; "
                        "2^18 is the library's default)")
    p.add_argument("--requests", type=int, default=2000, help="serving: requests per run")
    p.add_argument("--window", type=float, default=40.0, help="serving: longest arrival window per run (s)")
    p.add_argument("--no-companions", action="store_true",
                   help="large: leave out the shortened batching and serving comparisons added to the line")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="also run a plain 1 GiB device copy (reference for HBM traffic counters)")
    return p.parse_args()


PLAIN = {
    "mid": dict(n=1_000_000, m=10_000_000, gamma=2.1, wmax=5e4, gseed=2, k=6, cseed=12, samples=1_000_000,
                sseed=22, oracle_full=True, traffic="dp_mid_k6_hbm_traffic.txt", biased_lambda=0.02,
                label="mid: Chung-Lu n=1e6 m=1e7 exponent 2.1 w_max=5e4, k=6, zero-rooting"),
    "large": dict(n=4_000_000, m=60_000_000, gamma=2.3, wmax=2e5, gseed=3, k=8, cseed=13, samples=10_000_000,
                  sseed=23, oracle_scales=(256, 128), traffic="dp_large_k8_hbm_traffic.txt", biased_lambda=0.01,
                  label="large: Chung-Lu n=4e6 m=6e7 exponent 2.3 w_max=2e5, k=8, zero-rooting",
                  ags=dict(cbar=1000, round_size=100_000, budget=20_000_000, seed=33)),
}

ORACLE_SAMPLES = 200       # samples drawn (and classified) per timed oracle run
ORACLE_WORKERS_MAX = 16    # forked sampling workers of the all-core figure


def _oracle_rates(tab, g, k, sseed, workers):
    """Seconds per sample (draw + classification) of the oracle on one core, and
    with `workers` forked processes drawing disjoint index ranges of the same
    stream from the (inherited) table."""
    import multiprocessing as mp

    import oracle as O
    O.classify(g, k, tab.sample(1, seed=sseed)[0])          # per-k catalog, outside the timing
    t0 = time.perf_counter()
    v, _ = tab.sample(ORACLE_SAMPLES, seed=sseed)
    O.classify(g, k, v)
    one = (time.perf_counter() - t0) / ORACLE_SAMPLES

    def work(i, q):
        v, _ = tab.sample(ORACLE_SAMPLES, seed=sseed, first_index=i * ORACLE_SAMPLES)
        O.classify(g, k, v)
        q.put(i)

    ctx = mp.get_context("fork")
    q = ctx.Queue()
    t0 = time.perf_counter()
    ps = [ctx.Process(target=work, args=(i, q)) for i in range(workers)]
    for p in ps:
        p.start()
    for _ in ps:
        q.get()
    for p in ps:
        p.join()
    many = (time.perf_counter() - t0) / (workers * ORACLE_SAMPLES)
    return one, many


def cpu_baseline(cfg, full_m, samples):
    """The oracle, as is: its build (single-threaded: its DP has no parallel
    form) and its sampler + classification on one core and on all host cores
    (forked workers over disjoint sample indices). Runs before the GPU is
    touched. mid: on the bench's own input. large: the full build does not
    finish in the bench's time, so it is timed on two scaled graphs of the same
    family and extrapolated (labelled as such)."""
    import graphgen as gg
    import oracle as O
    k = cfg["k"]
    workers = max(1, min(os.cpu_count() or 1, ORACLE_WORKERS_MAX))
    if cfg.get("oracle_full"):
        g = gg.chung_lu(cfg["n"], cfg["m"], cfg["gamma"], cfg["wmax"], seed=cfg["gseed"])
        colors = gg.colors(g.n, k, seed=cfg["cseed"])
        t0 = time.perf_counter()
        tab = O.Table(g, colors, k, O.ROOT_ZERO)
        t_build = time.perf_counter() - t0
        one, many = _oracle_rates(tab, g, k, cfg["sseed"], workers)
        how = (f"measured on the bench's own input (Chung-Lu n={g.n}, m={g.m}, k={k}): build {t_build:.1f} s on one "
               f"core; {ORACLE_SAMPLES} samples + classification at {one * 1e3:.2f} ms/sample on one core, "
               f"{many * 1e3:.3f} ms/sample with {workers} forked workers (first {ORACLE_SAMPLES} indices of each "
               f"worker's range of the bench's stream)")
        extrapolated = False
    else:
        pts = []
        for scale in cfg["oracle_scales"]:
            n, m = cfg["n"] // scale, cfg["m"] // scale
            g = gg.chung_lu(n, m, cfg["gamma"], cfg["wmax"] / scale, seed=cfg["gseed"])
            colors = gg.colors(g.n, k, seed=cfg["cseed"])
            t0 = time.perf_counter()
            tab = O.Table(g, colors, k, O.ROOT_ZERO)
            tb = time.perf_counter() - t0
            one, many = _oracle_rates(tab, g, k, cfg["sseed"], workers)
            pts.append((scale, g.m, tb, one, many))
            del tab
        import math
        (s0, m0, b0, o0, y0), (s1, m1, b1, o1, y1) = pts
        # power laws in the edge count through the two measured scales
        eb = math.log(b1 / b0) / math.log(m1 / m0)
        eo = math.log(o1 / o0) / math.log(m1 / m0)
        ey = math.log(y1 / y0) / math.log(m1 / m0)
        f = full_m / m1
        t_build, one, many = b1 * f ** eb, o1 * f ** eo, y1 * f ** ey
        how = (f"EXTRAPOLATED: the oracle timed on Chung-Lu graphs of the same family at 1/{s0} and 1/{s1} scale "
               f"(m = {m0} and {m1}, w_max scaled alike, k={k}): build {b0:.2f} s and {b1:.2f} s on one core, "
               f"{ORACLE_SAMPLES} samples + classification at {o0 * 1e3:.2f} and {o1 * 1e3:.2f} ms/sample on one "
               f"core ({y0 * 1e3:.3f} and {y1 * 1e3:.3f} ms/sample with {workers} forked workers); each figure "
               f"extended to m = {full_m} by the power law through its two points (exponents build {eb:.2f}, "
               f"sample {eo:.2f}, all-core sample {ey:.2f}): build {t_build:.0f} s, {one * 1e3:.2f} ms/sample")
        extrapolated = True
    step1 = t_build + samples * one
    stepn = t_build + samples * many
    return {
        "value": samples / step1, "unit": "classified samples/s (table build + sampling + classification per step)",
        "cores": 1, "kind": "oracle", "extrapolated": extrapolated,
        "sample": how + f"; value = {samples} / (build + {samples} samples)",
        "build_s": t_build, "s_per_sample": one,
        "all_cores": {"value": samples / stepn, "cores": workers, "host_cpus": os.cpu_count(),
                      "s_per_sample": many,
                      "note": "build on one core (the oracle's DP is sequential), samples by forked workers"},
    }


def profile_fields(name):
    """Fields of a committed counter summary (profiles/<name>) when it was taken
    for the current DP and sampler sources, else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    csrc = os.path.join(ROOT, "paper_2009_03052_amd", "csrc")
    try:
        fields = {}
        for line in open(path):
            parts = line.split()
            if len(parts) >= 2:
                fields[parts[0]] = parts[1]
        h = hashlib.sha256()
        for f in ("dp.hip", "sample.hip", "device.hpp"):
            h.update(open(os.path.join(csrc, f), "rb").read())
        if fields.get("source_sha256") != h.hexdigest():
            return None
        return fields
    except OSError:
        return None


def round_skipping(scc, dg, dcol, k, ns, sseed, verts, par, zinfo, zbuild_ms):
    """The same graph and colouring with round skipping (balanced rooting, level
    k-1 skipped, stars sampled directly): build, shape-first uniform sampling and
    star sampling, next to the zero-rooting build of the plain step."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record()
    bt = scc.Table(dg, dcol, k, rooting=scc.ROOT_BALANCED, validate=False)
    ev[1].record()
    bt.sample(ns, seed=sseed, out=(verts, par))
    ev[2].record()
    bt.sample(ns, seed=sseed, shape=scc.star_shape(k), out=(verts, par))
    ev[3].record()
    torch.cuda.synchronize()
    bi = bt.info()
    star = scc.star_shape(k)
    u = lambda x: int(x[0]) | (int(x[1]) << 64)
    match = all(u(bi.tj[j]) == (0 if j == star else u(zinfo.tj[j])) for j in range(bi.num_unrooted))
    b_ms = ev[0].elapsed_time(ev[1])
    out = {"build_s": b_ms / 1e3, "zero_rooting_build_s": zbuild_ms / 1e3,
           "build_saving": 1 - b_ms / zbuild_ms if zbuild_ms > 0 else None,
           "table_bytes": int(bi.bytes), "zero_rooting_table_bytes": int(zinfo.bytes),
           "bytes_saving": 1 - bi.bytes / zinfo.bytes if zinfo.bytes else None,
           "level_ms": [round(bi.level_ms[h], 3) for h in range(1, k + 1)],
           "sample_per_s": ns / (ev[1].elapsed_time(ev[2]) / 1e3),
           "star_sample_per_s": ns / (ev[2].elapsed_time(ev[3]) / 1e3),
           "t_non_star": str(u(bi.t)), "stars": str(u(bi.stars)),
           "non_star_totals_equal_zero_rooting": match}
    del bt
    print(f"# round skipping: build {b_ms:.1f} ms vs {zbuild_ms:.1f} ms, {bi.bytes / 1e9:.2f} GB vs "
          f"{zinfo.bytes / 1e9:.2f} GB, totals match {match}", file=sys.stderr, flush=True)
    return out


def biased_colouring(scc, dg, k, lam, cseed, ns, sseed, verts, par, zinfo, zbuild_ms):
    """The same graph under a biased colouring (Sec. 3.5): colour 0 with
    probability 1 - (k-1) lambda, others lambda each; build, sampling, and the
    estimate t / p_k of the number of k-treelet copies next to the uniform one."""
    import torch
    dcol = scc.color_biased(dg.n, k, lam, seed=cseed)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record()
    bt = scc.Table(dg, dcol, k, rooting=scc.ROOT_ZERO, validate=False)
    ev[1].record()
    bt.sample(ns, seed=sseed, out=(verts, par))
    ev[2].record()
    torch.cuda.synchronize()
    bi = bt.info()
    u = lambda x: int(x[0]) | (int(x[1]) << 64)
    pb, pu = scc.colorful_probability(k, lam), scc.colorful_probability(k)
    b_ms = ev[0].elapsed_time(ev[1])
    est_b, est_u = u(bi.t) / pb, u(zinfo.t) / pu
    out = {"lambda": lam, "p_k": pb, "p_k_uniform": pu, "build_s": b_ms / 1e3, "uniform_build_s": zbuild_ms / 1e3,
           "table_bytes": int(bi.bytes), "uniform_table_bytes": int(zinfo.bytes),
           "sample_per_s": ns / (ev[1].elapsed_time(ev[2]) / 1e3), "t": str(u(bi.t)),
           "treelets_estimate": est_b, "uniform_treelets_estimate": est_u, "estimate_ratio": est_b / est_u}
    del bt
    print(f"# biased colouring lambda={lam}: build {b_ms:.1f} ms vs {zbuild_ms:.1f} ms, {bi.bytes / 1e9:.2f} GB vs "
          f"{zinfo.bytes / 1e9:.2f} GB, estimate ratio {est_b / est_u:.4f}", file=sys.stderr, flush=True)
    return out


def variable_length(scc, dg, dcol, k, ns, sseed, verts, par, zinfo):
    """The same table re-encoded with variable-length counts (Sec. 3.3): build
    (with the sampler's running sums, then the re-encoding), record bytes and
    sampling rate next to the fixed layout."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record()
    vt = scc.Table(dg, dcol, k, rooting=scc.ROOT_ZERO, vlc=True, validate=False)
    ev[1].record()
    vt.sample(ns, seed=sseed, out=(verts, par))
    ev[2].record()
    torch.cuda.synchronize()
    vi = vt.info()
    # the fixed layout here is already narrow (a u16 key and a 64-bit count for
    # most vertices); a layout of 16-bit keys and 128-bit counts throughout is
    # 18 bytes per stored count
    entries = sum(int(zinfo.nnz[h]) for h in range(2, k + 1))
    out = {"build_s": ev[0].elapsed_time(ev[1]) / 1e3, "record_bytes": int(vi.record_bytes),
           "fixed_record_bytes": int(zinfo.record_bytes),
           "record_saving": 1 - vi.record_bytes / zinfo.record_bytes if zinfo.record_bytes else None,
           "entries": entries,
           "saving_vs_128_bit_counts": 1 - vi.record_bytes / (18 * entries) if entries else None,
           "table_bytes": int(vi.bytes), "fixed_table_bytes": int(zinfo.bytes),
           "sample_per_s": ns / (ev[1].elapsed_time(ev[2]) / 1e3)}
    del vt
    print(f"# variable-length counts: build {out['build_s'] * 1e3:.1f} ms (with sampling preparation), records "
          f"{vi.record_bytes / 1e9:.2f} GB vs {zinfo.record_bytes / 1e9:.2f} GB", file=sys.stderr, flush=True)
    return out


def random_read_ceiling(scc, torch):
    """Device rate of reads of 64- and 128-byte records at random positions of a
    4 GiB zero-filled buffer (2^24 reads, best of 3): the neighbour-record
    gather's access pattern at the memory system's own limit, next to the
    8 TB/s sequential peak."""
    n_reads = 1 << 24
    buf = torch.zeros(1 << 29, dtype=torch.int64, device="cuda")
    out = {"buffer_bytes": buf.numel() * 8, "reads": n_reads}
    for rb in (64, 128):
        ms = min(scc.probe_random_reads(buf, rb, n_reads, salt=s) for s in range(3))
        out[f"GBs_{rb}B"] = n_reads * rb / ms / 1e6
        out[f"frac_of_peak_{rb}B"] = out[f"GBs_{rb}B"] / HBM_PEAK_GBS
    del buf
    torch.cuda.empty_cache()
    return out


def batching_instances():
    """16 colourings of a Chung-Lu graph (n=5e5, m~5e6, exponent 2.2, w_max=2.5e4) and 32
    uneven ER/BA graphs (n log-uniform in [1e3, 1e5], mean degree 4 + (i mod 17)); k = 5 + (i mod 3)."""
    import numpy as np

    import graphgen as gg
    out = []
    big = gg.chung_lu(500_000, 5_000_000, 2.2, 2.5e4, seed=4)
    for i in range(16):
        k = 5 + i % 3
        out.append((f"cl500k-c{i}", big, gg.colors(big.n, k, seed=100 + i), k))
    rng = np.random.default_rng(5)
    ns = np.exp(rng.uniform(np.log(1e3), np.log(1e5), 32)).astype(int)
    for i in range(32):
        d = 4 + i % 17
        n = int(ns[i])
        if i % 2 == 0:
            g = gg.erdos_renyi(n, n * d // 2, seed=5 + i)
        else:
            g = gg.barabasi_albert(n, (d + 1) // 2, seed=5 + i)
        k = 5 + (16 + i) % 3
        out.append((f"{'er' if i % 2 == 0 else 'ba'}{n}-d{d}", g, gg.colors(g.n, k, seed=200 + i), k))
    return out


def tables_equal_on_device(ta, tb, k):
    """Every stored level (offsets, keys, both count words) and the totals of two
    tables equal, compared on the device."""
    import torch
    if ta.totals() != tb.totals():
        return False
    for h in range(1, k + 1):
        xa, xb = ta.export_level(h, to_host=False), tb.export_level(h, to_host=False)
        if not all(x.shape == y.shape and torch.equal(x, y) for x, y in zip(xa, xb)):
            return False
    return True


def run_batching(a, emit=True):
    import torch

    import paper_2009_03052_amd as scc
    torch.cuda.set_device(0)
    raw = batching_instances()
    devg = {}
    inst = []
    for name, g, c, k in raw:
        if id(g) not in devg:
            devg[id(g)] = scc.DeviceGraph.from_graph(g)
        inst.append((devg[id(g)], torch.as_tensor(c).cuda(), k))
    print(f"# batching: {len(inst)} instances, {sum(g.n for _, g, _, _ in raw)} vertices", file=sys.stderr, flush=True)
    groups = {"colourings": inst[:16], "uneven_graphs": inst[16:], "all": inst}

    def plain(xs):
        for g, c, k in xs:
            t = scc.Table(g, c, k, validate=False)
            del t

    def batched(xs, plain_nnz=0):
        tabs, rep = scc.build_batch(xs, autotune=True, validate=False, plain_nnz=plain_nnz)
        del tabs
        return rep

    def timed(f, *args):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = f(*args)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    tuned = {}
    for name, xs in groups.items():
        plain(xs)
        tuned[name] = batched(xs)      # tunes once per batch shape (probes); later calls reuse the choice
        batched(xs, -1)
        r = tuned[name]
        print(f"# {name}: tuned tile={r['tile']} hub={r['hub_degree']} waves={r['waves']}", file=sys.stderr, flush=True)
    per = {}
    reps = []
    for name, xs in groups.items():
        tp, tb, tq = [], [], []
        for i in range(a.steps):
            tp.append(timed(plain, xs)[0])
            dt, rep = timed(batched, xs)
            tb.append(dt)
            tq.append(timed(batched, xs, -1)[0])
            if name == "all":
                reps.append(rep)
        per[name] = {"plain_s": sum(tp) / len(tp), "batched_s": sum(tb) / len(tb),
                     "persistent_only_s": sum(tq) / len(tq), "plain_instances": rep["plain_instances"]}
        per[name]["speedup_vs_plain"] = per[name]["plain_s"] / per[name]["batched_s"]
        print(f"# {name}: plain {per[name]['plain_s'] * 1e3:.1f} ms, batched {per[name]['batched_s'] * 1e3:.1f} ms "
              f"({rep['plain_instances']} instances on the level kernels), every instance in the persistent "
              f"launch {per[name]['persistent_only_s'] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    # full-size check: every batched table equals the plain build of its instance
    tabs, _ = scc.build_batch(inst, autotune=True, validate=False)
    equal = True
    for (g, c, k), bt in zip(inst, tabs):
        pt = scc.Table(g, c, k, validate=False)
        equal = equal and tables_equal_on_device(pt, bt, k)
        del pt
    del tabs
    print(f"# every batched table equals its plain build: {equal}", file=sys.stderr, flush=True)
    p_s, b_s = per["all"]["plain_s"], per["all"]["batched_s"]
    out = {
        "metric": "DP table build s & colorful-treelet samples/sec, batched/served vs plain",
        "value": len(inst) / b_s,
        "unit": "tables built per second (the batch scheduler: instances of at least 2^21 CSR entries on the "
                "level kernels, the rest in one persistent launch)",
        "n_gpus": 1, "steps": a.steps, "warmup": 1, "ms_per_step": b_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64/u128", "data": "synthetic",
        "config": {"workload": "batching: 16 colourings of Chung-Lu n=5e5 m=5e6 exponent 2.2 + 32 ER/BA graphs "
                               "n in [1e3, 1e5], k = 5..7, zero-rooting",
                   "instances": len(inst)},
        "plain_s": p_s, "batched_s": b_s, "speedup_vs_plain": p_s / b_s,
        "groups": per,
        "batched_tables_equal_plain": equal,
        "batch_report": {k: v for k, v in reps[-1].items() if k != "probes"},
        "tuning_probes": tuned["all"]["probes"],
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


SMALL_REQUEST = 1 << 14   # serving: requests of at most this many samples go first, whole
SMALL_STEP = 1 << 16      # serving: step size while a small request runs


def serving_tables():
    """Three Chung-Lu graphs, n = 2e6, m = 3e7, exponents 2.1 / 2.4 / 2.8, w_max = 1e5, k = 7."""
    import graphgen as gg
    out = []
    for i, gam in enumerate((2.1, 2.4, 2.8)):
        g = gg.chung_lu(2_000_000, 30_000_000, gam, 1e5, seed=6 + i)
        out.append((g, gg.colors(g.n, 7, seed=16 + i), 7))
        print(f"# serving graph {i}: n={g.n} m={g.m} d_max={int(g.degrees().max())}", file=sys.stderr, flush=True)
    return out


def serving_trace(count, seed=31):
    """Request mix: sizes log-uniform in [1e3, 1e6]; half uniform samples (classified) on a
    random graph, half AGS rounds from one client per graph; unit-mean exponential gaps."""
    import numpy as np
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(1e3), np.log(1e6), count)).astype(np.int64)
    ags = rng.random(count) < 0.5
    graph = rng.integers(0, 3, count)
    seeds = rng.integers(1, 1 << 40, count)
    gaps = rng.exponential(1.0, count)
    return [dict(n=int(sizes[i]), ags=bool(ags[i]), graph=int(graph[i]), seed=int(seeds[i]), gap=float(gaps[i]))
            for i in range(count)]


def drive(srv, trace, rate, sessions, window, keep_every=0):
    """Submits `trace` at Poisson arrival times (rate per second; rate = inf: all at once) from one
    thread, waits for and releases the results in order from another; returns the server's stats.
    keep_every > 0: the rows of every keep_every-th uniform request are copied out (st["kept"])."""
    import queue
    import threading
    q = queue.Queue()
    t0 = time.perf_counter()
    at = 0.0
    arrivals = []
    for r in trace:
        at += r["gap"] / rate if rate != float("inf") else 0.0
        arrivals.append(at)

    def submitter():
        for i, r in enumerate(trace):
            if arrivals[i] > window:
                break
            dt = arrivals[i] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            if r["ags"]:
                rid = srv.submit(r["graph"], r["n"], session=sessions[r["graph"]])
            else:
                rid = srv.submit(r["graph"], r["n"], seed=r["seed"], stream_id=i, classify=True)
            q.put((rid, "ags" if r["ags"] else "uniform", i))
        q.put(None)

    lat = {"uniform": [], "ags": []}
    by_size = {}
    kept = []

    def waiter():
        done = 0
        nu = 0
        while True:
            item = q.get()
            if item is None:
                break
            rid, kind, i = item
            keep = kind == "uniform" and keep_every > 0 and nu % keep_every == 0
            nu += kind == "uniform"
            r = srv.wait(rid, timeout=900.0, copy=keep)
            if keep:
                kept.append((i, r["verts"], r["parent"], r["cls"]))
            lat[kind].append(r["t_done"] - r["t_submit"])
            by_size.setdefault(size_bucket(trace[i]["n"]), []).append(r["t_done"] - r["t_submit"])
            srv.release(rid)
            done += 1
            if done % 250 == 0:
                print(f"#   {done} requests done", file=sys.stderr, flush=True)

    ts = [threading.Thread(target=submitter), threading.Thread(target=waiter)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    st = srv.stats()
    st["wall_s"] = time.perf_counter() - t0
    st["kept"] = kept
    for kind, xs in lat.items():
        xs = sorted(xs)
        if xs:
            st[f"{kind}_p50_ms"] = 1e3 * xs[max(0, int(0.5 * len(xs) + 0.5) - 1)]
            st[f"{kind}_p99_ms"] = 1e3 * xs[max(0, min(len(xs), int(0.99 * len(xs) + 0.5)) - 1)]
    st["samples_per_s"] = st["samples"] / st["span_s"] if st["span_s"] > 0 else 0.0
    st["by_size"] = {}
    for b, xs in sorted(by_size.items()):
        xs = sorted(xs)
        st["by_size"][b] = {"requests": len(xs), "p50_ms": 1e3 * xs[max(0, int(0.5 * len(xs) + 0.5) - 1)],
                            "p99_ms": 1e3 * xs[max(0, min(len(xs), int(0.99 * len(xs) + 0.5)) - 1)]}
    return st


def size_bucket(n):
    """Request-size bucket for latency reports: 1e3-1e4, 1e4-1e5, 1e5-1e6 samples."""
    return "1e3-1e4" if n < 10_000 else ("1e4-1e5" if n < 100_000 else "1e5-1e6")


K16 = dict(n=1 << 16, m=1 << 17, gamma=2.5, wmax=40.0, gseed=7, k=10, cseed=17, oracle_scale=64)


def run_k16(a):
    """The build for k up to 16 (sparse records keyed by DFS bitstring and
    colour set): whole builds timed, per-level terms and sort time, and the
    oracle on a graph of the same recipe 1/64 the size (time per vertex)."""
    cfg = K16
    import graphgen as gg
    base = None
    if not a.no_cpu_baseline:
        import oracle as O
        ns = cfg["n"] // cfg["oracle_scale"]
        gs = gg.chung_lu(ns, cfg["m"] // cfg["oracle_scale"], cfg["gamma"], cfg["wmax"], seed=cfg["gseed"])
        cs = gg.colors(gs.n, cfg["k"], seed=cfg["cseed"])
        t0 = time.perf_counter()
        ot = O.Table16(gs, cs, cfg["k"], O.ROOT_ZERO)
        o_s = time.perf_counter() - t0
        base = {"value": gs.n / o_s, "unit": "vertices per second (whole build)", "cores": 1, "kind": "oracle",
                "sample": f"the oracle's build of a Chung-Lu graph of the same recipe with n = {gs.n}, "
                          f"m = {gs.m} (1/{cfg['oracle_scale']} of the workload), k = {cfg['k']}: {o_s:.2f} s",
                "t": str(ot.total())}
        del ot
        print(f"# oracle: {o_s:.2f} s for n = {gs.n}", file=sys.stderr, flush=True)
    import torch

    import paper_2009_03052_amd as scc
    torch.cuda.set_device(0)
    n = cfg["n"] // 16 if a.small else cfg["n"]
    g = gg.chung_lu(n, cfg["m"] * n // cfg["n"], cfg["gamma"], cfg["wmax"], seed=cfg["gseed"])
    k = cfg["k"]
    colors = gg.colors(g.n, k, seed=cfg["cseed"])
    dg = scc.DeviceGraph.from_graph(g)
    dcol = torch.as_tensor(colors).cuda()
    print(f"# graph n={g.n} m={g.m} d_max={int(g.degrees().max())}, k={k}", file=sys.stderr, flush=True)
    for i in range(a.warmup):
        t = scc.Table16(dg, dcol, k, validate=False)
        del t
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(a.steps):
        t = scc.Table16(dg, dcol, k, validate=False)
        infos.append(t.info())
        total = t.total()
        del t
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    inf = infos[-1]
    prof = profile_fields16("k16_k10_hbm_traffic.txt")
    sort_ms = sum(inf.sort_ms[h] for h in range(1, k + 1))
    sort_b = sum(inf.sort_bytes[h] for h in range(1, k + 1))
    print(f"# timed {a.steps} builds: {dt * 1e3:.1f} ms/build, sorts {sort_ms:.1f} ms", file=sys.stderr, flush=True)
    out = {
        "metric": "DP table build s & colorful-treelet samples/sec, batched/served vs plain",
        "value": g.n / dt, "unit": f"vertices per second (whole k = {k} build, sparse records)",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u128", "data": "synthetic",
        "config": {"workload": f"k16: Chung-Lu n={g.n} m={g.m} exponent {cfg['gamma']} w_max={cfg['wmax']}, "
                               f"k={k}, zero-rooting, sparse records keyed by DFS bitstring",
                   "n": g.n, "m": g.m, "k": k},
        "build_s": dt, "t": str(total),
        "level_ms": [round(inf.level_ms[h], 3) for h in range(1, k + 1)],
        "sort_ms": [round(inf.sort_ms[h], 3) for h in range(1, k + 1)],
        "nnz": [int(inf.nnz[h]) for h in range(1, k + 1)],
        "terms": [int(inf.terms[h]) for h in range(1, k + 1)],
        "nbr_terms": [int(inf.nbr_terms[h]) for h in range(1, k + 1)],
        "table_bytes": int(inf.bytes), "peak_bytes": int(inf.peak_bytes),
        "roofline": {"bound": "hbm", "achieved": sort_b / (sort_ms * 1e6) if sort_ms > 0 else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": sort_b / (sort_ms * 1e6) / HBM_PEAK_GBS if sort_ms > 0 else None,
                     "traffic": float(prof["sort_traffic_bytes_per_build"]) if prof else None,
                     "traffic_gbs": (float(prof["sort_traffic_bytes_per_build"]) / (sort_ms * 1e6)
                                     if prof and sort_ms > 0 else None),
                     "traffic_unit": "HBM bytes per build of k16_hist + k16_scatter from TCC_EA0 requests",
                     "kernel": "radix sort of the terms (k16_hist, k16_scatter and their scans): 32 B per "
                               "element and pass", "bytes_per_build": sort_b, "ms_per_build": sort_ms},
    }
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


def run_serving(a, emit=True, modes=("continuous", "continuous_age10ms", "continuous_equal", "fifo")):
    import torch

    import paper_2009_03052_amd as scc
    torch.cuda.set_device(0)
    raw = serving_tables()
    tabs = []
    build_s = []
    for g, c, k in raw:
        dg = scc.DeviceGraph.from_graph(g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tabs.append(scc.Table(dg, torch.as_tensor(c).cuda(), k, rooting=scc.ROOT_ZERO, validate=False))
        torch.cuda.synchronize()
        build_s.append(time.perf_counter() - t0)
        print(f"# table built in {build_s[-1]:.3f} s, {tabs[-1].info().bytes / 1e9:.1f} GB", file=sys.stderr, flush=True)
    trace = serving_trace(a.requests)
    opts = dict(hbm_budget=24 << 30, step_samples=a.serve_step, chunk=4096, max_active=512)
    cbar = 1000

    def server(fifo, ags_weight=1.0, age_tau=0.0, small=False):
        extra = dict(small_request=SMALL_REQUEST, small_step=SMALL_STEP) if small else {}
        srv = scc.Server(tabs, fifo=fifo, ags_weight=ags_weight, age_tau=age_tau, **opts, **extra)
        sessions = [srv.ags_open(t, cbar=cbar, seed=900 + t, stream_id=t) for t in range(len(tabs))]
        return srv, sessions

    # saturated rates: a burst of the first requests, all submitted at once, in each mode
    sat = {}
    for name, fifo in (("continuous", False), ("fifo", True)):
        srv, sess = server(fifo, 1.0, 0.0, small=not fifo)
        sat[name] = drive(srv, trace[:min(300, len(trace))], float("inf"), sess, 1e9)["samples_per_s"]
        srv.close()
        print(f"# saturated {name}: {sat[name] / 1e6:.1f} M samples/s", file=sys.stderr, flush=True)
    burst = {"samples_per_s": sat["continuous"]}
    mean_n = sum(r["n"] for r in trace) / len(trace)
    sat_req = burst["samples_per_s"] / mean_n
    rate = 0.7 * sat_req
    print(f"# saturated: {burst['samples_per_s'] / 1e6:.1f} M samples/s = {sat_req:.1f} requests/s; "
          f"Poisson rate {rate:.1f}/s", file=sys.stderr, flush=True)
    res = {}
    # continuous: shares weighted by age (tau 10 ms), which bounds the tail of large
    # requests; the plain equal shares and heavier AGS rounds are reported beside it
    for name, fifo, aw, tau, small in (("continuous", False, 1.0, 0.0, True), ("continuous_age10ms", False, 1.0, 0.01, False),
                                       ("continuous_equal", False, 1.0, 0.0, False), ("fifo", True, 1.0, 0.0, False)):
        if name not in modes:
            continue
        srv, sess = server(fifo, aw, tau, small)
        res[name] = drive(srv, trace, rate, sess, a.window, keep_every=40 if name == "continuous" else 0)
        srv.close()
        r = res[name]
        print(f"# {name}: {r['completed']} requests, {r['samples_per_s'] / 1e6:.1f} M samples/s, "
              f"p50 {r['p50_ms']:.1f} ms, p99 {r['p99_ms']:.1f} ms; uniform p50/p99 "
              f"{r.get('uniform_p50_ms', 0):.1f}/{r.get('uniform_p99_ms', 0):.1f} ms, AGS rounds p50/p99 "
              f"{r.get('ags_p50_ms', 0):.1f}/{r.get('ags_p99_ms', 0):.1f} ms", file=sys.stderr, flush=True)
    c, f = res["continuous"], res["fifo"]
    # served rows equal scc_sample / scc_classify alone with the same arguments
    alone_equal = True
    for i, v, p, cl in c["kept"]:
        r = trace[i]
        t = tabs[r["graph"]]
        av, ap = t.sample(r["n"], seed=r["seed"], stream_id=i)
        _, acl = t.classify(av)
        alone_equal = alone_equal and torch.equal(av, v) and torch.equal(ap, p) and torch.equal(acl.view(torch.int32),
                                                                                              cl.view(torch.int32))
    print(f"# {len(c['kept'])} served requests equal scc_sample alone: {alone_equal}", file=sys.stderr, flush=True)
    keep = ("completed", "samples", "steps", "span_s", "samples_per_s", "p50_ms", "p99_ms", "mean_ms", "max_ms",
            "arena_peak", "uniform_p50_ms", "uniform_p99_ms", "ags_p50_ms", "ags_p99_ms", "by_size")
    out = {
        "metric": "DP table build s & colorful-treelet samples/sec, batched/served vs plain",
        "value": c["samples_per_s"], "unit": "samples/s served (continuous batching, small requests first, "
                                             "Poisson arrivals at 0.7x saturation, submission to completion)",
        "n_gpus": 1, "steps": c["completed"], "warmup": 0, "ms_per_step": c["mean_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64/u128", "data": "synthetic",
        "config": {"workload": "serving: 3 resident k=7 tables (Chung-Lu n=2e6 m=3e7, exponents 2.1/2.4/2.8, "
                               "w_max=1e5), requests of 1e3..1e6 samples (log-uniform), half uniform+classified, "
                               "half AGS rounds from 3 clients, Poisson arrivals",
                   "requests": len(trace), "arrival_rate_per_s": rate, "window_s": a.window},
        "table_build_s": build_s,
        "saturated_samples_per_s": sat["continuous"], "saturated_samples_per_s_fifo": sat["fifo"],
        "saturated_throughput_vs_fifo": sat["continuous"] / sat["fifo"] if sat["fifo"] > 0 else None,
        "continuous": {k: c[k] for k in keep}, "fifo": {k: f[k] for k in keep},
        "policy": f"small requests (<= {SMALL_REQUEST} samples) first and whole, then submission order; steps "
                  f"of {a.serve_step} samples, cut to {SMALL_STEP} while a small request runs",
        "served_equal_alone": alone_equal, "served_checked": len(c["kept"]),
        "p99_speedup_vs_fifo": f["p99_ms"] / c["p99_ms"] if c["p99_ms"] > 0 else None,
        "p50_speedup_vs_fifo": f["p50_ms"] / c["p50_ms"] if c["p50_ms"] > 0 else None,
        "throughput_vs_fifo": c["samples_per_s"] / f["samples_per_s"] if f["samples_per_s"] > 0 else None,
    }
    if "continuous_age10ms" in res:
        out["continuous_age_weighted_shares_10ms"] = {k: res["continuous_age10ms"][k] for k in keep}
    if "continuous_equal" in res:
        out["continuous_equal_shares"] = {k: res["continuous_equal"][k] for k in keep}
    del tabs
    if emit:
        print(json.dumps(out), flush=True)
    return out


def _u(x):
    return int(x[0]) | (int(x[1]) << 64)


def rooflines(tab, infos, k, samp_ms, ns, prof):
    """Roofline entries of the step: the DP join (gather of levels 1..k-1,
    combine of levels 2..k, level-k totals), its gather and combine parts, and
    the sampler. Bytes are algorithmic (from the stored record lengths), times
    the HIP-event durations of the timed builds (mean over steps)."""
    gb = tab.gather_bytes()
    cb, tb = tab.combine_bytes()
    mean = lambda f: sum(f(x) for x in infos) / len(infos)
    g_ms = mean(lambda x: sum(x.gather_ms[h] for h in range(2, k)))
    c_ms = mean(lambda x: sum(x.combine_ms[h] for h in range(2, k + 1)))
    j_ms = mean(lambda x: sum(x.level_ms[h] for h in range(1, k + 1)) + x.totals_ms)
    g_bytes = sum(gb[h] for h in range(2, k))
    c_bytes = sum(cb[h] for h in range(2, k + 1))
    j_bytes = sum(gb[h] for h in range(1, k)) + c_bytes + tb

    def entry(bytes_, ms, kernel, traffic_key=None):
        ach = bytes_ / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        tr = float(prof[traffic_key]) if (prof and traffic_key and traffic_key in prof) else None
        out = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
               "traffic": tr, "kernel": kernel, "bytes_per_build": bytes_, "ms_per_build": ms}
        if tr is not None and ms > 0:
            # what the memory system moved: the counters' bytes over the same duration
            out["traffic_gbs"] = tr / (ms * 1e-3) / 1e9
            out["traffic_frac"] = out["traffic_gbs"] / HBM_PEAK_GBS
        return out

    join = entry(j_bytes, j_ms, "DP join: k_gather1, k_gather*, k_hub_prepare, k_combine*, k_words, scans, k_pack, "
                 "k_totals and scans (every level of the build plus the level-k totals)", "traffic_bytes_per_build")
    join["traffic_unit"] = "HBM bytes per build from TCC_EA0 read requests by size (32/64/128 B) and write requests"
    parts = {
        "gather": entry(g_bytes, g_ms, "neighbour-sum gather of levels 2..k-1 (k_gather_group, k_gather_list, "
                        "k_gather, k_gather_wide, k_gather_hub, k_hub_prepare)", "gather_traffic_bytes_per_build"),
        "combine": entry(c_bytes, c_ms, "combine of levels 2..k with compaction and packing (k_combine*, "
                         "k_combine_list, k_combine_wide, k_words, scans, k_pack)", "combine_traffic_bytes_per_build"),
    }
    sp = {"bound": "hbm random access", "samples_per_s": ns / (samp_ms / 1e3) if samp_ms > 0 else 0.0,
          "ms_per_launch": samp_ms, "kernel": "k_sample"}
    if prof and "sampler_read_bytes_per_sample" in prof:
        bps = float(prof["sampler_read_bytes_per_sample"])
        sp.update({"hbm_read_bytes_per_sample": bps, "achieved": bps * ns / (samp_ms * 1e-3) / 1e9,
                   "peak": HBM_PEAK_GBS, "unit": "GB/s"})
        sp["frac"] = sp["achieved"] / HBM_PEAK_GBS
        if "sampler_l2_request_bytes_per_sample" in prof:
            sp["l2_request_bytes_per_sample"] = float(prof["sampler_l2_request_bytes_per_sample"])
    else:
        sp.update({"hbm_read_bytes_per_sample": None, "achieved": None, "frac": None})
    parts["sampler"] = sp
    return join, parts


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if a.workload == "batching":
        return run_batching(a)
    if a.workload == "serving":
        return run_serving(a)
    if a.workload == "k16":
        return run_k16(a)
    cfg = PLAIN[a.workload]
    base = None
    if not a.no_cpu_baseline and not a.small:
        # first, while no GPU context exists (its sampling workers are forked)
        print("# cpu baseline (the oracle) ...", file=sys.stderr, flush=True)
        base = cpu_baseline(cfg, cfg["m"], a.samples if a.samples is not None else cfg["samples"])
        print(f"# cpu baseline: {base['value']:.1f} samples/s on 1 core", file=sys.stderr, flush=True)
    import torch

    import graphgen as gg
    import paper_2009_03052_amd as scc

    torch.cuda.set_device(0)
    if a.calibrate_copy:
        # a plain copy of known size: reads and writes 2^30 bytes each; the ratio of
        # these to what the read / write request counters report scales them
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print("# calibration copy of 1073741824 bytes done", file=sys.stderr, flush=True)
    if a.small:
        g = gg.chung_lu(cfg["n"] // 10, cfg["m"] // 10, cfg["gamma"], cfg["wmax"] / 10, seed=cfg["gseed"])
    else:
        g = gg.chung_lu(cfg["n"], cfg["m"], cfg["gamma"], cfg["wmax"], seed=cfg["gseed"])
    k = cfg["k"]
    colors = gg.colors(g.n, k, seed=cfg["cseed"])
    dg = scc.DeviceGraph.from_graph(g)
    dcol = torch.as_tensor(colors).cuda()
    ns = a.samples if a.samples is not None else cfg["samples"]
    sseed = cfg["sseed"]
    verts = torch.empty((ns, k), dtype=torch.int32, device="cuda")
    par = torch.empty((ns, k), dtype=torch.int8, device="cuda")
    code = torch.empty(ns, dtype=torch.int32, device="cuda")
    cls = torch.empty(ns, dtype=torch.int32, device="cuda")
    print(f"# graph n={g.n} m={g.m} d_max={int(g.degrees().max())}", file=sys.stderr, flush=True)

    def step():
        tab = scc.Table(dg, dcol, k, rooting=scc.ROOT_ZERO, validate=False)
        tab.sample(ns, seed=sseed, out=(verts, par))
        tab.classify(verts, out=(code, cls))
        return tab

    for i in range(a.warmup):
        tab = step()
        del tab
        print(f"# warmup {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(a.steps):
        tab = step()
        infos.append(tab.info())
        del tab
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    print(f"# timed {a.steps} steps: {dt * 1e3:.1f} ms/step", file=sys.stderr, flush=True)

    # phase split (one extra step, events around each call)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    tab = scc.Table(dg, dcol, k, rooting=scc.ROOT_ZERO, validate=False)
    ev[1].record()
    tab.sample(ns, seed=sseed, out=(verts, par))
    ev[2].record()
    tab.classify(verts, out=(code, cls))
    ev[3].record()
    torch.cuda.synchronize()
    build_ms, samp_ms, cls_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])
    info = tab.info()
    prof = profile_fields(cfg["traffic"])
    join, parts = rooflines(tab, infos, k, samp_ms, ns, prof)
    print(f"# DP join {join['achieved']:.0f} GB/s ({join['frac']:.3f} of peak); gather "
          f"{parts['gather']['achieved']:.0f} GB/s, combine {parts['combine']['achieved']:.0f} GB/s",
          file=sys.stderr, flush=True)
    ags = None
    if "ags" in cfg and not a.no_round_skipping:
        A = cfg["ags"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = tab.ags(cbar=A["cbar"], round_size=A["round_size"], budget=A["budget"], seed=A["seed"])
        torch.cuda.synchronize()
        t_ags = time.perf_counter() - t0
        drawn = int(r["n_j"].sum())
        ags = {"cbar": A["cbar"], "round_size": A["round_size"], "budget": A["budget"],
               "rounds": int(len(r["round_shapes"])), "samples": drawn, "seconds": t_ags,
               "samples_per_s": drawn / t_ags if t_ags > 0 else 0.0,
               "classes_hit": int((r["hits"] > 0).sum()), "classes_covered": int((r["hits"] >= A["cbar"]).sum()),
               "shapes_used": sorted(set(int(x) for x in r["round_shapes"]))}
        print(f"# AGS: {ags['rounds']} rounds, {drawn} samples in {t_ags:.2f} s", file=sys.stderr, flush=True)
    rs = None if a.no_round_skipping else round_skipping(scc, dg, dcol, k, ns, sseed, verts, par, info, build_ms)
    bc = None if a.no_round_skipping else biased_colouring(scc, dg, k, cfg["biased_lambda"], cfg["cseed"], ns, sseed,
                                                           verts, par, info, build_ms)
    vl = None if a.no_round_skipping else variable_length(scc, dg, dcol, k, ns, sseed, verts, par, info)
    rr = None if a.no_round_skipping else random_read_ceiling(scc, torch)
    if rr:
        print(f"# random reads: {rr['GBs_64B']:.0f} GB/s (64 B), {rr['GBs_128B']:.0f} GB/s (128 B)", file=sys.stderr,
              flush=True)
    out = {
        "metric": "DP table build s & colorful-treelet samples/sec, batched/served vs plain",
        "value": ns / dt,
        "unit": "classified samples/s (table build + sampling + classification per step)",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64/u128",
        "data": "synthetic",
        "config": {"workload": cfg["label"] + f", {ns} uniform samples + classification",
                   "n": g.n, "m": g.m, "d_max": int(g.degrees().max()), "k": k, "samples": ns},
        "build_s": build_ms / 1e3, "sample_per_s": ns / (samp_ms / 1e3), "classify_per_s": ns / (cls_ms / 1e3),
        "level_ms": [round(info.level_ms[h], 3) for h in range(1, k + 1)],
        "gather_ms": [round(info.gather_ms[h], 3) for h in range(1, k)],
        "combine_ms": [round(info.combine_ms[h], 3) for h in range(2, k + 1)],
        "totals_ms": round(info.totals_ms, 3),
        "wide_vertices": [int(info.wide_vertices[h]) for h in range(1, k + 1)],
        "wide_input_rows": [[int(x) for x in info.wide_input_rows[h]] for h in range(1, k + 1)],
        "lane_width_test_levels": [h for h in range(1, k + 1) if info.lane_width_test >> h & 1],
        "table_bytes": int(info.bytes), "t": str(_u(info.t)),
        "roofline": join,
        "roofline_parts": parts,
    }
    if rr is not None:
        out["random_read_ceiling"] = rr
    if ags is not None:
        out["ags"] = ags
    if rs is not None:
        out["round_skipping"] = rs
    if bc is not None:
        out["biased_colouring"] = bc
    if vl is not None:
        out["variable_length_counts"] = vl
    if base is not None:
        out["cpu_baseline"] = base
    if a.workload == "large" and not a.no_round_skipping and not a.no_companions and not a.small:
        # the batched and served forms beside the plain one, shortened (the full runs are
        # --workload batching and --workload serving)
        del tab, dg, dcol, verts, par, code, cls
        torch.cuda.empty_cache()
        out["batched_vs_plain"] = companion_batching(a)
        torch.cuda.empty_cache()
        out["served_vs_fifo"] = companion_serving(a)
    print(json.dumps(out), flush=True)


def companion_batching(a):
    """The batching workload, three timed steps per group."""
    b = run_batching(argparse.Namespace(**{**vars(a), "steps": 3}), emit=False)
    g = b["groups"]
    return {"plain_s": b["plain_s"], "batched_s": b["batched_s"], "speedup_vs_plain": b["speedup_vs_plain"],
            "colourings_speedup_vs_plain": g["colourings"]["speedup_vs_plain"],
            "uneven_graphs_speedup_vs_plain": g["uneven_graphs"]["speedup_vs_plain"],
            "batched_tables_equal_plain": b["batched_tables_equal_plain"], "steps": 3,
            "workload": b["config"]["workload"]}


def companion_serving(a):
    """The serving workload's trace, continuous batching (small requests first) against
    first-in first-out only."""
    r = run_serving(argparse.Namespace(**{**vars(a), "requests": 2000, "window": 40.0}), emit=False,
                    modes=("continuous", "fifo"))
    c, f = r["continuous"], r["fifo"]
    return {"continuous_p50_ms": c["p50_ms"], "continuous_p99_ms": c["p99_ms"],
            "fifo_p50_ms": f["p50_ms"], "fifo_p99_ms": f["p99_ms"],
            "p50_speedup_vs_fifo": r["p50_speedup_vs_fifo"], "p99_speedup_vs_fifo": r["p99_speedup_vs_fifo"],
            "saturated_samples_per_s": r["saturated_samples_per_s"],
            "saturated_throughput_vs_fifo": r["saturated_throughput_vs_fifo"],
            "served_equal_alone": r["served_equal_alone"], "served_checked": r["served_checked"],
            "requests_submitted": r["config"]["requests"], "completed": c["completed"],
            "window_s": r["config"]["window_s"], "workload": r["config"]["workload"]}


# ---------------------------------------------------------------------------
# Summaries of rocprofv3 output (what profiles/ holds):
#   python bench.py summarise trace <run_kernel_trace.csv>
#   python bench.py summarise counters <label> <samples per k_sample> <dir of the read pass> <dir of the write pass>
#   python bench.py summarise sq <dir of SQ pass 1> <dir of SQ pass 2>
# ---------------------------------------------------------------------------
def _short_kernel(name):
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name[:name.index("(")].strip() if "(" in name else name.strip()


def _first_build(names):
    """Indices of the first table build: from its first kernel to the last one before
    the first sampling call's preparation (per-edge colours, hub running sums built
    apart from the build) or, without one, before the first k_sample."""
    start = next(i for i, nm in enumerate(names) if nm in ("k_row_lists", "k_validate_rows"))
    prep = ("k_sample", "k_edge_colours", "k_hub_info", "k_hub_index", "k_hubpre_chunk")
    end = next(i for i, nm in enumerate(names) if i > start and nm in prep)
    return start, end


def summarise_trace(path):
    import csv
    import collections
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    names = [_short_kernel(r["Kernel_Name"]) for r in rows]
    a, b = _first_build(names)
    build = rows[a:b]
    t0 = int(build[0]["Start_Timestamp"])
    t1 = max(int(r["End_Timestamp"]) for r in build)
    dur = lambda r: int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    busy = sum(dur(r) for r in build)
    agg = collections.defaultdict(lambda: [0, 0])
    for r, nm in zip(build, names[a:b]):
        agg[nm][0] += 1
        agg[nm][1] += dur(r)
    print(f"one build (the first): {(t1 - t0) / 1e6:.1f} ms from its first kernel to the end of its last, "
          f"kernels busy {busy / 1e6:.1f} ms\n")
    print("| kernel (one build) | calls | ms | % of busy |\n|---|---|---|---|")
    for nm, (c, d) in sorted(agg.items(), key=lambda x: -x[1][1]):
        if d >= 0.001 * busy:
            print(f"| {nm} | {c} | {d / 1e6:.2f} | {100 * d / busy:.1f} |")
    print()
    for want in ("k_sample", "k_classify"):
        ds = [dur(r) for r, nm in zip(rows, names) if nm == want]
        if ds:
            print(f"{want}: {len(ds)} calls, average {sum(ds) / len(ds) / 1e6:.3f} ms")


def _counter_dispatches(d):
    import csv
    import collections
    import glob
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not f:
        raise SystemExit(f"no counter_collection.csv under {d}")
    disp = collections.OrderedDict()
    for r in csv.DictReader(open(f[0])):
        e = disp.setdefault(int(r["Dispatch_Id"]), {"name": _short_kernel(r["Kernel_Name"]), "c": {}})
        e["c"][r["Counter_Name"]] = e["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [disp[i] for i in sorted(disp)]


def summarise_counters(label, ns, dir_a, dir_b):
    """HBM bytes per kernel of one build from the TCC_EA0 request counters: reads
    32 RDREQ_32B + 64 RDREQ_64B + 128 RDREQ_128B (pass A), writes
    32 (WRREQ - WRREQ_64B) + 64 WRREQ_64B (pass B), calibrated on the 1 GiB copy."""
    import collections
    import hashlib
    A, B = _counter_dispatches(dir_a), _counter_dispatches(dir_b)
    rd = lambda c: (32 * c.get("TCC_EA0_RDREQ_32B_sum", 0) + 64 * c.get("TCC_EA0_RDREQ_64B_sum", 0)
                    + 128 * c.get("TCC_EA0_RDREQ_128B_sum", 0))
    wr = lambda c: (32 * (c.get("TCC_EA0_WRREQ_sum", 0) - c.get("TCC_EA0_WRREQ_64B_sum", 0))
                    + 64 * c.get("TCC_EA0_WRREQ_64B_sum", 0))

    def calib(ds, f):   # the copy: the largest pre-build dispatch
        best = None
        for d in ds:
            if d["name"].startswith("k_"):
                break
            if best is None or f(d["c"]) > best[1]:
                best = (d["name"], f(d["c"]))
        return best

    def cls(nm):
        if (nm.startswith("k_gather") and nm != "k_gather_bytes") or nm == "k_hub_prepare":
            return "gather"
        if nm.startswith("k_combine") or nm.startswith("k_pack") or nm == "k_words":
            return "combine"
        return "other"

    ca, cb = calib(A, rd), calib(B, wr)
    na, nb = [d["name"] for d in A], [d["name"] for d in B]
    (a0, a1), (b0, b1) = _first_build(na), _first_build(nb)
    ba, bb = A[a0:a1], B[b0:b1]
    if [d["name"] for d in ba] != [d["name"] for d in bb]:
        raise SystemExit("the two passes dispatched different kernels")
    tot = collections.defaultdict(lambda: [0.0, 0.0, 0, 0.0])
    for da, db in zip(ba, bb):
        t = tot[da["name"]]
        t[0] += rd(da["c"])
        t[1] += wr(db["c"])
        t[2] += 1
        t[3] += db["c"].get("TCC_EA0_RDREQ_DRAM_sum", 0)
    g = collections.defaultdict(lambda: [0.0, 0.0])
    for nm, t in tot.items():
        g[cls(nm)][0] += t[0]
        g[cls(nm)][1] += t[1]
    sa = [d for d in A if d["name"] == "k_sample"]
    sb = [d for d in B if d["name"] == "k_sample"]
    h = hashlib.sha256()
    for f in ("dp.hip", "sample.hip", "device.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2009_03052_amd", "csrc", f), "rb").read())
    print(f"workload: {label}")
    print(f"calibration copy (1073741824 bytes each way): read requests by size give {ca[1]:.0f} bytes ({ca[0]}), "
          f"write requests {cb[1]:.0f} bytes ({cb[0]})")
    print("per kernel of one build (HBM-side TCC_EA0 requests; DRAM rdreq = TCC_EA0_RDREQ_DRAM, requests):")
    print(f"  {'kernel':28s} {'dispatches':>10s} {'read MB':>12s} {'write MB':>12s}  {'DRAM rdreq':>12s}")
    for nm, t in sorted(tot.items(), key=lambda x: -(x[1][0] + x[1][1])):
        print(f"  {nm:28s} {t[2]:10d} {t[0] / 1e6:12.1f} {t[1] / 1e6:12.1f}  {t[3]:12.0f}")
    for key in ("gather", "combine", "other"):
        print(f"{key}_read_bytes_per_build {g[key][0]:.0f}\n{key}_write_bytes_per_build {g[key][1]:.0f}")
    print(f"traffic_bytes_per_build {sum(x[0] + x[1] for x in g.values()):.0f}")
    print(f"gather_traffic_bytes_per_build {g['gather'][0] + g['gather'][1]:.0f}")
    print(f"combine_traffic_bytes_per_build {g['combine'][0] + g['combine'][1]:.0f}")
    print(f"sampler_dispatches {len(sa)}")
    print(f"sampler_read_bytes_per_sample {sum(rd(d['c']) for d in sa) / (ns * max(1, len(sa))):.1f}")
    print(f"sampler_write_bytes_per_sample {sum(wr(d['c']) for d in sb) / (ns * max(1, len(sb))):.1f}")
    print(f"source_sha256 {h.hexdigest()}  (dp.hip + sample.hip + device.hpp at the time of the counter runs)")


def summarise_counters16(label, dir_a, dir_b):
    """HBM bytes per kernel of one k <= 16 build (every k16_* dispatch of the run),
    from the same request counters as summarise_counters."""
    import collections
    import hashlib
    A, B = _counter_dispatches(dir_a), _counter_dispatches(dir_b)
    rd = lambda c: (32 * c.get("TCC_EA0_RDREQ_32B_sum", 0) + 64 * c.get("TCC_EA0_RDREQ_64B_sum", 0)
                    + 128 * c.get("TCC_EA0_RDREQ_128B_sum", 0))
    wr = lambda c: (32 * (c.get("TCC_EA0_WRREQ_sum", 0) - c.get("TCC_EA0_WRREQ_64B_sum", 0))
                    + 64 * c.get("TCC_EA0_WRREQ_64B_sum", 0))
    ba = [d for d in A if d["name"].startswith("k16_")]
    bb = [d for d in B if d["name"].startswith("k16_")]
    if [d["name"] for d in ba] != [d["name"] for d in bb]:
        raise SystemExit("the two passes dispatched different kernels")
    tot = collections.defaultdict(lambda: [0.0, 0.0, 0])
    for da, db in zip(ba, bb):
        t = tot[da["name"]]
        t[0] += rd(da["c"])
        t[1] += wr(db["c"])
        t[2] += 1
    h = hashlib.sha256(open(os.path.join(ROOT, "paper_2009_03052_amd", "csrc", "dp16.hip"), "rb").read())
    print(f"workload: {label}")
    print("per kernel of one build (HBM-side TCC_EA0 requests):")
    print(f"  {'kernel':28s} {'dispatches':>10s} {'read MB':>12s} {'write MB':>12s}")
    for nm, t in sorted(tot.items(), key=lambda x: -(x[1][0] + x[1][1])):
        print(f"  {nm:28s} {t[2]:10d} {t[0] / 1e6:12.1f} {t[1] / 1e6:12.1f}")
    sort = sum(t[0] + t[1] for nm, t in tot.items() if nm in ("k16_hist", "k16_scatter"))
    print(f"traffic_bytes_per_build {sum(t[0] + t[1] for t in tot.values()):.0f}")
    print(f"sort_traffic_bytes_per_build {sort:.0f}  (k16_hist + k16_scatter)")
    print(f"source_sha256 {h.hexdigest()}  (dp16.hip at the time of the counter runs)")


def summarise_sq(dir_1, dir_2):
    """Per kernel of the first build and its first sampler launch: the shader
    sequencer's wave counters summed over dispatches, per wave. SQ_WAVE_CYCLES and
    SQ_WAIT_ANY count in the counters' own cycle unit; their ratio is the share of a
    wave's lifetime spent waiting (on memory, LDS or a barrier)."""
    import collections
    agg = collections.defaultdict(collections.Counter)
    for d in (dir_1, dir_2):
        ds = _counter_dispatches(d)
        names = [e["name"] for e in ds]
        a, b = _first_build(names)
        for e in ds[a:b + 1]:
            agg[e["name"]].update(e["c"])
    print("| kernel | waves | cycles / wave | waiting | VALU instr / wave | SALU | LDS instr | VMEM reads | "
          "LDS bank-conflict cycles / wave |")
    print("|---|---|---|---|---|---|---|---|---|")
    for nm, c in sorted(agg.items(), key=lambda x: -x[1]["SQ_WAVE_CYCLES"]):
        w = c["SQ_WAVES"] or 1.0
        if c["SQ_WAVE_CYCLES"] < 1e9:
            continue
        wait = c["SQ_WAIT_ANY"] / c["SQ_WAVE_CYCLES"] if c["SQ_WAVE_CYCLES"] else 0.0
        print(f"| {nm} | {c['SQ_WAVES']:.3g} | {c['SQ_WAVE_CYCLES'] / w:.0f} | {100 * wait:.0f} % | "
              f"{c['SQ_INSTS_VALU'] / w:.0f} | {c['SQ_INSTS_SALU'] / w:.0f} | {c['SQ_INSTS_LDS'] / w:.0f} | "
              f"{c['SQ_INSTS_VMEM_RD'] / w:.0f} | {c['SQ_LDS_BANK_CONFLICT'] / w:.0f} |")


def profile_fields16(name):
    """Fields of profiles/<name> when taken for the current dp16.hip, else None."""
    import hashlib
    try:
        fields = {}
        for line in open(os.path.join(ROOT, "profiles", name)):
            parts = line.split()
            if len(parts) >= 2:
                fields[parts[0]] = parts[1]
        h = hashlib.sha256(open(os.path.join(ROOT, "paper_2009_03052_amd", "csrc", "dp16.hip"), "rb").read())
        return fields if fields.get("source_sha256") == h.hexdigest() else None
    except OSError:
        return None


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "summarise" and sys.argv[2] == "counters16":
        summarise_counters16(sys.argv[3], sys.argv[4], sys.argv[5])
    elif len(sys.argv) > 2 and sys.argv[1] == "summarise" and sys.argv[2] == "trace":
        summarise_trace(sys.argv[3])
    elif len(sys.argv) > 2 and sys.argv[1] == "summarise" and sys.argv[2] == "counters":
        summarise_counters(sys.argv[3], int(sys.argv[4]), sys.argv[5], sys.argv[6])
    elif len(sys.argv) > 2 and sys.argv[1] == "summarise" and sys.argv[2] == "sq":
        summarise_sq(sys.argv[3], sys.argv[4])
    else:
        main()
