"""Benchmark: the whole hot path on the mid workload, on one MI355X.

One step = table build (Eq. (1) DP, all levels, totals) + 10^6 uniform
colourful 6-treelet samples + their classification, on a Chung-Lu graph with
n = 10^6, m = 10^7, exponent 2.1, maximum expected degree 5e4 (seeded), k = 6,
zero-rooting. The graph and colours are resident in HBM before timing starts.

Prints one JSON line. `value` is classified samples per second of whole steps
(build included). The dominant kernel is the neighbour-record gather of the DP
(HBM-bound); its roofline entry divides the algorithmic bytes of the gather
launches by their duration measured with HIP events on the build's stream.
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
    p.add_argument("--samples", type=int, default=1_000_000)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--small", action="store_true", help="small graph (for quick checks)")
    p.add_argument("--workload", default="mid", choices=["mid", "batching"],
                   help="mid (default): the plain method on the mid graph; batching: 48 instances, plain vs one batched launch")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="also run a plain 1 GiB device copy (reference for HBM traffic counters)")
    return p.parse_args()


def cpu_baseline(full_m, samples):
    """The oracle, as is, on a bounded sample of the workload (single thread)."""
    import graphgen as gg
    import oracle as O
    scale = 8
    n, m = 1_000_000 // scale, 10_000_000 // scale
    g = gg.chung_lu(n, m, 2.1, 5e4 / scale, seed=2)
    colors = gg.colors(g.n, 6, seed=12)
    t0 = time.perf_counter()
    tab = O.Table(g, colors, 6, O.ROOT_ZERO)
    t_build = time.perf_counter() - t0
    ns = 300
    t0 = time.perf_counter()
    v, _ = tab.sample(ns, seed=22)
    O.classify(g, 6, v)
    t_samp = (time.perf_counter() - t0) / ns
    est_step = t_build * (full_m / g.m) + samples * t_samp
    return {
        "value": samples / est_step, "unit": "samples/s", "cores": 1, "kind": "oracle",
        "sample": (f"oracle build on a 1/{scale}-scale graph of the same family (Chung-Lu n={n}, m={g.m}, "
                   f"exponent 2.1, w_max={5e4 / scale:.0f}) took {t_build:.2f} s, scaled by edges to m={full_m}; "
                   f"sampling+classification {t_samp * 1e3:.2f} ms/sample measured on {ns} samples of that table; "
                   f"value = {samples} / (scaled build + {samples} samples)"),
    }


def measured_traffic():
    """HBM bytes per step of the gather kernels from the committed counter summary,
    or None when the gather source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "gather_mid_k6_hbm_traffic.txt")
    src = os.path.join(ROOT, "paper_2009_03052_amd", "csrc", "dp.hip")
    try:
        fields = {}
        for line in open(path):
            parts = line.split()
            if len(parts) >= 2:
                fields[parts[0]] = parts[1]
        cur = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if fields.get("source_sha256") != cur:
            return None
        return float(fields["traffic_bytes_per_step"])
    except (OSError, KeyError, ValueError):
        return None


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


def run_batching(a):
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

    def plain():
        for g, c, k in inst:
            t = scc.Table(g, c, k)
            del t

    def batched():
        tabs, rep = scc.build_batch(inst, autotune=True)
        del tabs
        return rep

    plain()
    rep0 = batched()      # tunes once (probes), later calls reuse the choice
    print(f"# tuned: tile={rep0['tile']} hub={rep0['hub_degree']} probes={rep0['probes']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tp = []
    tb = []
    reps = []
    for i in range(a.steps):
        torch.cuda.synchronize(); t0 = time.perf_counter(); plain(); torch.cuda.synchronize()
        tp.append(time.perf_counter() - t0)
        t0 = time.perf_counter(); reps.append(batched()); torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
    p_s, b_s = sum(tp) / len(tp), sum(tb) / len(tb)
    out = {
        "metric": "DP table build s & colorful-treelet samples/sec, batched/served vs plain",
        "value": len(inst) / b_s, "unit": "tables built per second (one batched launch for all 48 instances)",
        "n_gpus": 1, "steps": a.steps, "warmup": 1, "ms_per_step": b_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64/u128", "data": "synthetic",
        "config": {"workload": "batching: 16 colourings of Chung-Lu n=5e5 m=5e6 exponent 2.2 + 32 ER/BA graphs "
                               "n in [1e3, 1e5], k = 5..7, zero-rooting",
                   "instances": len(inst)},
        "plain_s": p_s, "batched_s": b_s, "speedup_vs_plain": p_s / b_s,
        "batch_report": {k: v for k, v in reps[-1].items() if k != "probes"},
        "tuning_probes": rep0["probes"],
    }
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if a.workload == "batching":
        return run_batching(a)
    import torch

    import graphgen as gg
    import paper_2009_03052_amd as scc

    torch.cuda.set_device(0)
    if a.calibrate_copy:
        # a plain copy of known size: reads and writes 2^30 bytes each; the ratio of
        # these to what FETCH_SIZE / WRITE_SIZE report for it scales the counters
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print("# calibration copy of 1073741824 bytes done", file=sys.stderr, flush=True)
    if a.small:
        g = gg.chung_lu(100_000, 1_000_000, 2.1, 5e3, seed=2)
    else:
        g = gg.chung_lu(1_000_000, 10_000_000, 2.1, 5e4, seed=2)
    k = 6
    colors = gg.colors(g.n, k, seed=12)
    dg = scc.DeviceGraph.from_graph(g)
    dcol = torch.as_tensor(colors).cuda()
    ns = a.samples
    verts = torch.empty((ns, k), dtype=torch.int32, device="cuda")
    par = torch.empty((ns, k), dtype=torch.int8, device="cuda")
    code = torch.empty(ns, dtype=torch.int32, device="cuda")
    cls = torch.empty(ns, dtype=torch.int32, device="cuda")
    print(f"# graph n={g.n} m={g.m} d_max={int(g.degrees().max())}", file=sys.stderr, flush=True)

    def step():
        tab = scc.Table(dg, dcol, k, rooting=scc.ROOT_ZERO)
        tab.sample(ns, seed=22, out=(verts, par))
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
    tab = scc.Table(dg, dcol, k, rooting=scc.ROOT_ZERO)
    ev[1].record()
    tab.sample(ns, seed=22, out=(verts, par))
    ev[2].record()
    tab.classify(verts, out=(code, cls))
    ev[3].record()
    torch.cuda.synchronize()
    build_ms, samp_ms, cls_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])
    info = tab.info()

    # gather launches of the timed builds: HIP-event durations recorded on the
    # build's stream; algorithmic bytes are the same for every build of the input
    gms = [sum(x.gather_ms[h] for h in range(2, k)) for x in infos]
    g_ms = sum(gms) / len(gms)
    gb = tab.gather_bytes()
    g_bytes = sum(gb[h] for h in range(2, k))
    achieved = g_bytes / (g_ms * 1e-3) / 1e9 if g_ms > 0 else 0.0
    traffic = measured_traffic()
    out = {
        "metric": "DP table build s & colorful-treelet samples/sec, batched/served vs plain",
        "value": ns / dt,
        "unit": "classified samples/s (table build + sampling + classification per step)",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64/u128",
        "data": "synthetic",
        "config": {"workload": "mid: Chung-Lu n=1e6 m=1e7 exponent 2.1 w_max=5e4, k=6, zero-rooting, "
                               f"{ns} uniform samples + classification",
                   "n": g.n, "m": g.m, "d_max": int(g.degrees().max()), "k": k, "samples": ns},
        "build_s": build_ms / 1e3, "sample_per_s": ns / (samp_ms / 1e3), "classify_per_s": ns / (cls_ms / 1e3),
        "level_ms": [round(info.level_ms[h], 3) for h in range(1, k + 1)],
        "table_bytes": int(info.bytes), "t": str(int(info.t[0]) | (int(info.t[1]) << 64)),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "bytes per step (4 gather launches), FETCH_SIZE x2.0 + WRITE_SIZE x1.0",
                     "kernel": "k_gather + k_gather_hub (neighbour-record gather of the DP, levels 2..k-1)",
                     "bytes_per_step": g_bytes, "ms_per_step": g_ms},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g.m, ns)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
