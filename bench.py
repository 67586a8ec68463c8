#!/usr/bin/env python3
"""Throughput and latency of the LST chain on one MI355X (plain per-event path).

One step = the whole chain (hit bucketing, MD, LS, T3, T5, T5 duplicate
removal, pLS, pT3/pT5, duplicate removal and cross-cleaning into track
candidates) for one PU200-like event with pixel seeds, inputs already
resident in HBM, synchronous (lst_build_event returns after the device work
and the counter read-back).  Events cycle through a pool of distinct seeded
events.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--pool P] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
WORKLOAD = {
    "pu200_seeded": ("PU200-like synthetic event with pixel seeds: 6 barrel layers (|z|<120 cm) + 2x5 endcap "
                     "disks of 10x5 cm bi-layer pT modules (19,262 modules), 8,000 helices pT 0.8-50 GeV "
                     "|eta|<2.4 + 40,000 loopers pT 0.1-0.8 GeV + 5% noise (~5.0e5 outer hits), ~8.9k pixel "
                     "seeds (10% fake); FP32 coordinates, int32 indices"),
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=40)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--pool", type=int, default=8, help="distinct events cycled through")
    p.add_argument("--workload", default="pu200_seeded", choices=sorted(WORKLOAD))
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--cpu-events", type=int, default=1, help="events in the CPU-baseline sample")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic bytes per launch of a launch site: the distinct inputs the launch
# must read once and the outputs it must write once, from the record sizes of
# the device layout: hit 16 B (x, y, z, r); MD 36 B (hit pair 8, module 4,
# anchor 16, stub 8); LS 16 B (MD pair 8, angles 8); T3 40 B (MDs 16, attrs
# 16, first anchor 8); T5 68 B (T3 pair 8, MDs 20, attrs 32, keep 4, first
# anchor 4 of 8); pLS 32 B; pT entry 24 B (seed/object 8, attrs 16);
# direction 16 B; count / offset / flag words 4 B.  c = object counts.
def algorithmic_bytes(site, c, n_outer, n_mod, n_edges, n_seeds, n_tc):
    md, ls, t3, t5, p3, p5 = c["md"], c["ls"], c["t3"], c["t5"], c["pt3"], c["pt5"]
    S, M, E = n_seeds, n_mod, n_edges
    n0, n1, n2 = c.get("tc0", 0), c.get("tc1", 0), c.get("tc2", 0)
    hit_in = 16 * n_outer + 8 * 2 * M          # bucketed hits + bucket offsets
    md_in = 28 * md                             # anchor + stub + module of every MD
    table = {
        "md_count": hit_in + 20 * M + 4 * M,
        "md_fill": hit_in + 20 * M + 4 * (M + 1) + 36 * md,
        "ls_count": md_in + 8 * (M + 1) + 4 * E + 4 * M + 4 * md,
        "ls_fill": md_in + 8 * (M + 1) + 4 * E + 4 * M + 4 * (md + 1) + 16 * ls,
        "t3_count": 8 * ls + 20 * md + 4 * (md + 1) + 4 * ls,
        "t3_fill": 8 * ls + 20 * md + 4 * (md + 1) + 4 * (ls + 1) + 40 * t3,
        "t5_count": 32 * t3 + 20 * md + 4 * (md + 1) + 4 * (ls + 1) + 4 * t3,
        "t5_fill": 32 * t3 + 20 * md + 4 * (md + 1) + 4 * (ls + 1) + 4 * (t3 + 1) + 60 * t5,
        "t5_dedup": 60 * t5 + 8 * md + 4 * (md + 1) + 20 * t5 + 12 * t5,
        "pt3_count": 32 * S + 8 * t3 + 4 * S,
        "pt3_fill": 32 * S + 8 * t3 + 4 * (S + 1) + 24 * p3,
        "pt5_count": 32 * S + 12 * t5 + 4 * S,
        "pt5_fill": 32 * S + 12 * t5 + 4 * (S + 1) + 24 * p5,
        "tc_pt3": 16 * p3 + 32 * S + 4 * S + 16 * n0 + 4 * p3,
        "tc_t5": 8 * t5 + 16 * t5 + 16 * (n0 + n1) + 4 * t5,
        "tc_pls": 8 * S + 32 * S + 16 * (n0 + n1 + n2) + 4 * S,
        "tc_write": 4 * (p5 + p3 + t5 + S) * 2 + 4 * (14 * n0 + 10 * (n1 + n2)) + 4 * n_tc * 3,
    }
    return table.get(site)


def main():
    args = parse()
    if args.gpus != 1:
        log(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported "
            "(events are independent; multi-GPU sharding by event is described in DESIGN.md)")
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2207_08207_amd as lst
    from lstgen import make_event
    from lstgen.events import geometry_for

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    geom = geometry_for(args.workload)
    g = lst.Geometry(geom)
    log(f"bench: generating {args.pool} {args.workload} events")
    pool, host = [], []
    for i in range(args.pool):
        ev = make_event(args.workload, i)
        host.append(ev)
        pool.append(lst.upload_event(ev, dev))
    n_hits_max = max(e.n_hits for e in host)
    n_seeds_max = max(e.n_seeds for e in host)
    cap = lst.lst_default_capacity(n_hits_max, n_seeds_max)
    ws = torch.empty(lst.lst_workspace_bytes(g.handle, n_hits_max, n_seeds_max, cap), dtype=torch.uint8, device=dev)
    log(f"bench: workspace {ws.numel() / 2**20:.1f} MiB, max hits {n_hits_max}, max seeds {n_seeds_max}")

    def step(i, timed_site=None):
        st, h = lst.lst_build_event(g.handle, pool[i % len(pool)], ws, cap, stream)
        if st != lst.LST_OK:
            raise lst.LSTError(st, lst.lst_last_error())
        t = lst.lst_get_site_time(h) if timed_site is not None else None
        counts, _ = lst.lst_get_stage_counts(h)
        lst.lst_release_event(h)
        return counts, t

    # find the dominant launch site (per-site HIP-event timing on two events, outside the timed region)
    sites = lst.lst_kernel_sites()
    per_site = np.zeros(len(sites))
    for k in range(len(sites)):
        lst.lst_set_timed_site(k)
        for i in range(2):
            per_site[k] += step(i, k)[1]
    lst.lst_set_timed_site(-1)
    dom = int(np.argmax(per_site))
    log("bench: site ms (2 events): " + ", ".join(f"{sites[k]}={per_site[k] / 2:.3f}"
                                                  for k in np.argsort(-per_site)[:8]))
    for i in range(args.warmup):
        step(i)
    # timed region: K synchronous steps; the dominant site is bracketed by HIP events
    lst.lst_set_timed_site(dom)
    torch.cuda.synchronize()
    lat, dom_ms, counts_all = [], [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        s0 = time.perf_counter()
        counts, t = step(args.warmup + i, dom)
        lat.append(time.perf_counter() - s0)
        dom_ms.append(t)
        counts_all.append(counts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lst.lst_set_timed_site(-1)
    value = args.steps / elapsed
    lat_ms = np.array(lat) * 1e3
    # roofline of the dominant kernel: algorithmic bytes per launch / measured launch time
    ev_of = [host[(args.warmup + i) % len(host)] for i in range(args.steps)]
    nb = []
    for ev, c in zip(ev_of, counts_all):
        cc = dict(md=int(c[0]), ls=int(c[1]), t3=int(c[2]), t5=int(c[3]), pt3=int(c[5]), pt5=int(c[6]))
        nb.append(algorithmic_bytes(sites[dom], cc, int((ev.module >= 0).sum()), geom.n_modules,
                                    int(geom.map_targets.size), ev.n_seeds, int(c[7])))
    roof = None
    if all(b is not None for b in nb):
        avg_bytes = float(np.mean(nb))
        avg_s = float(np.mean(dom_ms)) / 1e3
        ach = avg_bytes / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": sites[dom], "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None,
                "bytes_per_launch": int(avg_bytes), "launch_ms": round(avg_s * 1e3, 4)}
    out = {
        "metric": "events/s + p50/p99 event latency, PU200-like synthetic, plain per-event path, 1 GPU",
        "value": round(value, 3), "unit": "events/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOAD[args.workload], "events_in_pool": args.pool,
                   "mean_hits": int(np.mean([e.n_hits for e in host])),
                   "mean_seeds": int(np.mean([e.n_seeds for e in host])), "form": "plain synchronous per event"},
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                       "p99": round(float(np.percentile(lat_ms, 99)), 3)},
        "roofline": roof,
    }
    if not args.no_cpu:
        import oracle
        og = oracle.OracleGeometry(geom)
        t = time.perf_counter()
        for i in range(args.cpu_events):
            oracle.run(og, host[i])
        cpu_s = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(args.cpu_events / cpu_s, 4), "unit": "events/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{args.cpu_events} {args.workload} event(s) (seed 3000..), full chain, "
                                         f"serial FP32 C oracle, {cpu_s:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
