#!/usr/bin/env python3
"""Throughput and latency of the LST chain on one MI355X: served vs plain.

Every event goes through the whole chain (hit bucketing, MD, LS, T3, T5, T5
duplicate removal, pLS, pT3/pT5, duplicate removal and cross-cleaning into
track candidates), inputs already resident in HBM.  One step = one full
round of the server: streams x max-batch events (8 x 32 = 256 by default),
so K steps time 256 K events.  Forms measured:

* served (the headline `value`): the library's serving loop (streams x
  batches) with the K rounds' PU200-like seeded events available at once;
  the headline latency is the served p50 / p99 of the Poisson trace below;
* plain: synchronous lst_build_event per event, one at a time;
* e2e: plain, but from pinned host arrays: host-to-device copy, the chain,
  and the track candidates copied back (the PCIe-inclusive rate);
* trace: an open-loop Poisson trace (500 events/s, pile-up U[50, 250])
  through the server and through the plain FIFO path (1 stream, batch 1),
  plus a sweep of offered rates;
* batched: a captured hipGraph plan over B slots (pile-up U[140, 250]).

The CPU baseline runs the serial C oracle on one event per host core, all
cores at once.

Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--pool P] [--no-cpu] ...
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
LAUNCH_SHAPES = os.path.join(ROOT, "paper_2207_08207_amd", "launch_shapes_mi355x.json")
PMC_TRAFFIC = os.path.join(ROOT, "paper_2207_08207_amd", "pmc_traffic_mi355x.json")


def measured_traffic(site):
    """HBM bytes per event of a launch site from the recorded FETCH_SIZE / WRITE_SIZE runs, scaled by
    the reference copy kernel, or None when there is no record for it or the kernels changed since."""
    import hashlib
    try:
        with open(PMC_TRAFFIC) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_2207_08207_amd", "csrc", f), "rb").read()
                   for f in ("lst_kernels.hip", "lst_select.hpp", "lst_ws.hpp"))
    if rec.get("site") != site or rec.get("kernel_sources_sha256_16") != hashlib.sha256(src).hexdigest()[:16]:
        return None
    return rec
WORKLOAD = {
    "pu200_seeded": ("PU200-like synthetic event with pixel seeds: 6 barrel layers (|z|<120 cm) + 2x5 endcap "
                     "disks of 10x5 cm bi-layer pT modules (19,262 modules), 8,000 helices pT 0.8-50 GeV "
                     "|eta|<2.4 + 40,000 loopers pT 0.1-0.8 GeV + 5% noise (~5.0e5 outer hits), ~8.9k pixel "
                     "seeds (10% fake); FP32 coordinates, int32 indices"),
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=16,
                   help="server rounds timed (one round = streams x max-batch events)")
    p.add_argument("--warmup", type=int, default=2, help="untimed server rounds before the timed ones")
    p.add_argument("--pool", type=int, default=12, help="distinct events cycled through")
    p.add_argument("--streams", type=int, default=8,
                   help="server streams (8 x 32 measured 3,259 ev/s on one box against 3,060-3,138 for 8 x 16, "
                        "3,095 for 12 x 16 and 3,028 for 16 x 8)")
    p.add_argument("--max-batch", type=int, default=32, help="events per server launch sequence")
    p.add_argument("--rate", type=float, default=500.0, help="Poisson arrival rate of the trace [events/s]")
    p.add_argument("--trace", type=int, default=1000, help="requests in the open-loop trace (0: skip)")
    p.add_argument("--sweep", default="100,200,500,1000,2000",
                   help="offered rates of the served-vs-plain rate sweep [events/s] (empty: skip)")
    p.add_argument("--batch", type=int, default=64, help="slots of the captured batched plan (0: skip)")
    p.add_argument("--forms", default="plain,plain_graph,stub16,ext,displaced,e2e,served,trace,batched,copy,probe",
                   help="comma list of forms to run (served is the headline and always runs)")
    p.add_argument("--site", default=None,
                   help="launch site to time for the roofline (default: the largest in a per-site calibration)")
    p.add_argument("--workload", default="pu200_seeded", choices=sorted(WORKLOAD))
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--no-physics", action="store_true",
                   help="skip the truth-matched efficiency / fake / duplicate rates of the pool events")
    p.add_argument("--launch-config", default=LAUNCH_SHAPES,
                   help="JSON launch shapes to load (the packaged MI355X tuning; 'none' for the defaults)")
    p.add_argument("--tune", type=int, default=0,
                   help="autotune the launch shapes on this many pool events before any form (0: load instead)")
    p.add_argument("--save-launch-config", default=None, help="write the launch shapes used to this JSON file")
    p.add_argument("--cpu-workers", type=int, default=0,
                   help="oracle processes run side by side for the CPU baseline (0: the host's cores, at most 16)")
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
        "pt_count": 32 * S + 8 * t3 + 12 * t5 + 8 * S,
        "pt3_fill": 32 * S + 8 * t3 + 4 * (S + 1) + 24 * p3,
        "pt5_fill": 32 * S + 12 * t5 + 4 * (S + 1) + 24 * p5,
        "tc_pt3": 16 * p3 + 32 * S + 4 * S + 16 * n0 + 4 * p3,
        "tc_t5": 8 * t5 + 16 * t5 + 16 * (n0 + n1) + 4 * t5,
        "tc_pls": 8 * S + 32 * S + 16 * (n0 + n1 + n2) + 4 * S,
        "tc_write": 4 * (p5 + p3 + t5 + S) * 2 + 4 * (14 * n0 + 10 * (n1 + n2)) + 4 * n_tc * 3,
    }
    return table.get(site)


# The stages of the whole chain, each reading its inputs once and writing its
# outputs once (the fills, which read what their count pass read and write the
# objects; duplicate removal; cleaning; the TC write).  Their sum plus the hit
# bucketing (16 B raw read + 20 B bucketed write per hit) is the chain's
# algorithmic bytes per event; the count passes' re-reads are not counted.
CHAIN_SITES = ("md_fill", "ls_fill", "t3_fill", "t5_fill", "t5_dedup", "pt3_fill", "pt5_fill",
               "tc_pt3", "tc_t5", "tc_pls", "tc_write")


def chain_bytes(c, n_hits, n_outer, n_mod, n_edges, n_seeds):
    """Algorithmic bytes of one event through the whole chain (c = stage counts MD..TC)."""
    cc = dict(md=int(c[0]), ls=int(c[1]), t3=int(c[2]), t5=int(c[3]), pt3=int(c[5]), pt5=int(c[6]))
    tot = 16 * n_hits + 20 * n_outer
    for site in CHAIN_SITES:
        tot += algorithmic_bytes(site, cc, n_outer, n_mod, n_edges, n_seeds, int(c[7]))
    return tot


def percentiles(x_ms):
    import numpy as np
    x = np.asarray(x_ms, float)
    return {"p50": round(float(np.percentile(x, 50)), 3), "p99": round(float(np.percentile(x, 99)), 3)}


def run_trace(lst, g, dev, n_streams, max_batch, pool_bytes, arrivals, ids):
    """Open-loop replay: request i (event ids[i]) arrives at arrivals[i] on the server clock."""
    srv = lst.Server(g, n_streams, max_batch, pool_bytes)
    # warm-up: every stream runs full batches once before the timed trace
    n_warm = n_streams * max_batch * 2
    for i in range(n_warm):
        srv.submit(dev[ids[i % len(ids)]], -1 - i, 0.0)
    srv.drain(n_warm, lambda r: lst.lst_release_event(r["event"]) if r["event"] else None, timeout_s=300.0)
    t0 = srv.now() + 0.05
    for i, (a, k) in enumerate(zip(arrivals, ids)):
        srv.submit(dev[k], i, t0 + a)
    lat, done, first_arr = [], [], t0
    bad = []

    def take(r):
        if r["status"] != lst.LST_OK:
            bad.append(r["status"])
        lat.append((r["done_s"] - r["arrival_s"]) * 1e3)
        done.append(r["done_s"])
        if r["event"]:
            lst.lst_release_event(r["event"])

    srv.drain(len(arrivals), take, timeout_s=300.0)
    srv.close()
    if bad:
        raise RuntimeError(f"served requests failed with statuses {sorted(set(bad))}")
    span = max(done) - first_arr
    return lat, len(arrivals) / span


def _make(spec):
    from lstgen import make_event
    return make_event(*spec)


def make_events(specs):
    """Generated events for [(config, number), ...], made in parallel processes (CPU only)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    n = max(1, min(16, len(os.sched_getaffinity(0)), len(specs)))
    with ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_make, specs))


def _oracle_worker(workload, ev, start, out):
    """One CPU-baseline process: build the oracle's geometry, wait for the start signal, run one event."""
    try:
        import oracle
        from lstgen.events import geometry_for
        og = oracle.OracleGeometry(geometry_for(workload))
        out.put(("ready", 0.0))
        start.wait()
        t = time.perf_counter()
        r = oracle.run(og, ev)
        out.put(("done", (time.perf_counter() - t, r.step_seconds())))
    except BaseException as e:  # report instead of leaving the parent waiting
        out.put(("error", repr(e)))


def cpu_baseline(workload, events, n_workers):
    """Oracle throughput on the host: n_workers processes, one event each, started together."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    start, out = ctx.Event(), ctx.Queue()
    procs = [ctx.Process(target=_oracle_worker, args=(workload, events[i % len(events)], start, out))
             for i in range(n_workers)]
    for p in procs:
        p.start()
    def get(what):
        import queue
        t_end = time.time() + 600
        while True:
            try:
                m = out.get(timeout=2)
                break
            except queue.Empty:
                dead = [p.exitcode for p in procs if p.exitcode not in (None, 0)]
                if dead or time.time() > t_end:
                    start.set()
                    raise RuntimeError(f"oracle worker exited with {dead[0]}" if dead else "oracle workers timed out")
        if m[0] != what:
            start.set()
            raise RuntimeError(f"oracle worker: {m}")
        return m[1]

    for _ in procs:
        get("ready")
    t0 = time.perf_counter()
    start.set()
    done = [get("done") for _ in procs]
    wall = time.perf_counter() - t0
    for p in procs:
        p.join()
        if p.exitcode != 0:
            raise RuntimeError(f"oracle worker exited with {p.exitcode}")
    # each worker is one serial event on one core: median wall seconds of every step
    import numpy as np
    steps = {k: round(float(np.median([d[1][k] for d in done])), 4) for k in done[0][1]}
    return n_workers / wall, wall, sorted(d[0] for d in done), steps


def main():
    args = parse()
    if args.gpus != 1:
        log(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported "
            "(events are independent: several GPUs would each serve their own share of the events)")
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
    host = make_events([(args.workload, i) for i in range(args.pool)])
    pool = [lst.upload_event(ev, dev) for ev in host]
    n_hits_max = max(e.n_hits for e in host)
    n_seeds_max = max(e.n_seeds for e in host)
    cap = lst.lst_default_capacity(n_hits_max, n_seeds_max)
    ws_one = lst.lst_workspace_bytes(g.handle, n_hits_max, n_seeds_max, cap)
    ws = torch.empty(ws_one, dtype=torch.uint8, device=dev)
    log(f"bench: workspace {ws.numel() / 2**20:.1f} MiB per event, max hits {n_hits_max}, max seeds {n_seeds_max}")

    def step(i, timed_site=None, gh=None):
        st, h = lst.lst_build_event(g.handle if gh is None else gh, pool[i % len(pool)], ws, cap, stream)
        if st != lst.LST_OK:
            raise lst.LSTError(st, lst.lst_last_error())
        t = lst.lst_get_site_time(h) if timed_site is not None else None
        counts, _ = lst.lst_get_stage_counts(h)
        lst.lst_release_event(h)
        return counts, t

    # ---- launch shapes: autotuned on a batch of pool events, or loaded; used by every form
    tuned = None
    if args.tune > 0:
        t0 = time.perf_counter()
        res = g.autotune(pool[:min(args.tune, len(pool))], reps=2)
        tuned = {k: v[0] for k, v in res.items()}
        log(f"bench: autotuned in {time.perf_counter() - t0:.1f} s: {tuned}")
    elif args.launch_config != "none" and os.path.exists(args.launch_config):
        g.load_launch_config(args.launch_config)
        tuned = g.launch_config()
        log(f"bench: launch shapes from {args.launch_config}: {tuned}")
    if args.save_launch_config:
        g.save_launch_config(args.save_launch_config)
    forms = set(args.forms.split(","))
    sites = lst.lst_kernel_sites()
    if args.site is not None:
        dom = sites.index(args.site)
    else:
        # dominant launch site: per-site HIP-event timing on two events (outside the timed regions)
        per_site = np.zeros(len(sites))
        for k in range(len(sites)):
            lst.lst_set_timed_site(k)
            for i in range(2):
                per_site[k] += step(i, k)[1]
        lst.lst_set_timed_site(-1)
        dom = int(np.argmax(per_site))
        log("bench: site ms (2 events): " + ", ".join(f"{sites[k]}={per_site[k] / 2:.3f}"
                                                      for k in np.argsort(-per_site)))
        log(f"bench: sum of site times {per_site.sum() / 2:.3f} ms per event")

    n_outer = [int((ev.module >= 0).sum()) for ev in host]

    def event_bytes(k, c):
        cc = dict(md=int(c[0]), ls=int(c[1]), t3=int(c[2]), t5=int(c[3]), pt3=int(c[5]), pt5=int(c[6]))
        return algorithmic_bytes(sites[dom], cc, n_outer[k], geom.n_modules, int(geom.map_targets.size),
                                 host[k].n_seeds, int(c[7]))

    # ---- served at saturation (the headline), measured first so that its pool is allocated like a
    # server's at start-up: every request available at once; the dominant launch site of every
    # batched launch sequence is bracketed by HIP events on its stream
    n_streams, max_batch = args.streams, args.max_batch
    round_events = n_streams * max_batch
    pool_bytes = int(ws_one * (round_events + 2))
    srv = lst.Server(g, n_streams, max_batch, pool_bytes)
    n_warm = max(1, args.warmup) * round_events
    for i in range(n_warm):
        srv.submit(pool[i % len(pool)], -1 - i, 0.0)
    srv.drain(n_warm, lambda r: lst.lst_release_event(r["event"]))
    lst.lst_set_timed_site(dom)
    n_served = args.steps * round_events
    results = []

    def take(r):
        # only what the result handle holds; the byte bookkeeping runs after the timed region
        c, _ = lst.lst_get_stage_counts(r["event"])
        results.append((r["id"], r["arrival_s"], r["admit_s"], r["done_s"], lst.lst_get_site_time(r["event"]), c))
        lst.lst_release_event(r["event"])

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tnow = srv.now()
    for i in range(n_served):
        srv.submit(pool[i % len(pool)], i, tnow)
    srv.drain(n_served, take)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lst.lst_set_timed_site(-1)
    srv.close()
    del srv  # its pool (a whole round of workspaces) goes back to the device before the other forms
    torch.cuda.empty_cache()
    value = n_served / elapsed
    served_lat, launches, chain_served = [], {}, []
    for rid, arr, adm, done, ms, c in results:
        served_lat.append((done - arr) * 1e3)
        k = rid % len(host)
        rec = launches.setdefault(adm, [ms, 0.0])
        b = event_bytes(k, c)
        rec[1] = None if (b is None or rec[1] is None) else rec[1] + b
        chain_served.append(chain_bytes(c, host[k].n_hits, n_outer[k], geom.n_modules, int(geom.map_targets.size),
                                        host[k].n_seeds))
    log(f"bench: served {value:.1f} events/s over {n_served} events ({args.steps} rounds of {n_streams} streams x "
        f"{max_batch} per batch, {len(launches)} launch sequences)")

    # ---- plain: synchronous per event
    plain = None
    if "plain" in forms:
        for i in range(max(args.warmup, 4)):
            step(i)
        torch.cuda.synchronize()
        lat = []
        n_plain = 32
        t0 = time.perf_counter()
        for i in range(n_plain):
            s0 = time.perf_counter()
            step(4 + i)
            lat.append((time.perf_counter() - s0) * 1e3)
        torch.cuda.synchronize()
        plain_elapsed = time.perf_counter() - t0
        plain = {"events_per_s": round(n_plain / plain_elapsed, 3), "latency_ms": percentiles(lat),
                 "events": n_plain}
        log(f"bench: plain {plain}")

    # ---- displaced muons (5 cm cube) with the impact-parameter bound widened to 3.6 cm
    displaced = None
    if "displaced" in forms:
        from lstgen.truth_metrics import pooled_metrics
        g_d = lst.Geometry(geom)
        if tuned:
            g_d.set_launch_config(tuned)
        g_d.set_impact_bound(3.6)
        cube = [make_event("cube", k) for k in range(40)]
        cube_dev = [lst.upload_event(e, dev) for e in cube]
        for d in cube_dev[:4]:
            lst.run_event(g_d, d).close()
        torch.cuda.synchronize()
        pairs = []
        t0 = time.perf_counter()
        for e, d in zip(cube, cube_dev):
            r = lst.run_event(g_d, d)
            pairs.append((e, r.track_candidates()))
            r.close()
        el = time.perf_counter() - t0
        m = pooled_metrics(pairs)
        displaced = {"workload": "cube: 50 muons per event from vertices uniform in a 5 cm cube, 200 noise hits",
                     "impact_bound_cm": 3.6, "events": len(cube),
                     "events_per_s_with_readback": round(len(cube) / el, 2),
                     "efficiency": round(m["efficiency"], 5), "fake_rate": round(m["fake_rate"], 5),
                     "efficiency_vs_dxy": [(lo, hi, n, None if e is None else round(e, 4))
                                           for lo, hi, n, e in m["efficiency_vs_dxy"]]}
        log(f"bench: displaced {displaced}")

    # ---- one event per replay of a captured one-slot plan (the chain as one HIP graph):
    # per-event latency without the launch overhead of ~70 separate kernel launches
    plain_graph = None
    if "plain_graph" in forms:
        plan1 = lst.Plan(g, 1, n_hits_max, n_seeds_max)
        for i in range(max(args.warmup, 4)):
            for r in plan1.run([pool[i % len(pool)]]):
                r.close()
        torch.cuda.synchronize()
        n_pg = 32
        lat = []
        t0 = time.perf_counter()
        for i in range(n_pg):
            s0 = time.perf_counter()
            for r in plan1.run([pool[(4 + i) % len(pool)]]):
                r.close()
            lat.append((time.perf_counter() - s0) * 1e3)
        torch.cuda.synchronize()
        plain_graph = {"events_per_s": round(n_pg / (time.perf_counter() - t0), 3), "latency_ms": percentiles(lat),
                       "events": n_pg, "form": "one event per replay of a captured one-slot plan"}
        plan1.close()
        del plan1
        log(f"bench: plain graph {plain_graph}")

    # ---- plain with the MD stubs stored in binary16 (the half-precision storage variant)
    stub16 = None
    if "stub16" in forms:
        g_h = lst.Geometry(geom)
        if tuned:
            g_h.set_launch_config(tuned)
        g_h.set_stub_precision(16)
        for i in range(max(args.warmup, 4)):
            step(i, gh=g_h.handle)
        torch.cuda.synchronize()
        n_h = 32
        lat = []
        t0 = time.perf_counter()
        for i in range(n_h):
            s0 = time.perf_counter()
            step(4 + i, gh=g_h.handle)
            lat.append((time.perf_counter() - s0) * 1e3)
        torch.cuda.synchronize()
        stub16 = {"events_per_s": round(n_h / (time.perf_counter() - t0), 3), "latency_ms": percentiles(lat),
                  "events": n_h}
        k = sites.index("ls_count")
        lst.lst_set_timed_site(k)
        stub16["ls_count_ms"] = round(sum(step(i, k, gh=g_h.handle)[1] for i in range(4)) / 4, 4)
        lst.lst_set_timed_site(-1)
        log(f"bench: plain with binary16 MD stubs {stub16}")

    # ---- plain with the track-extension step at the end of the chain
    ext = None
    if "ext" in forms:
        g_ext = lst.Geometry(geom)
        if tuned:
            g_ext.set_launch_config(tuned)
        g_ext.set_track_extensions(True)
        for i in range(max(args.warmup, 4)):
            step(i, gh=g_ext.handle)
        torch.cuda.synchronize()
        n_ext = 32
        lat = []
        t0 = time.perf_counter()
        for i in range(n_ext):
            s0 = time.perf_counter()
            step(4 + i, gh=g_ext.handle)
            lat.append((time.perf_counter() - s0) * 1e3)
        torch.cuda.synchronize()
        ext = {"events_per_s": round(n_ext / (time.perf_counter() - t0), 3), "latency_ms": percentiles(lat),
               "events": n_ext, "step": "the chain plus the track-extension step, one event at a time"}
        site_ms = {}
        for name in ("tc_ext", "tc_ext_scan", "tc_ext_write"):
            k = sites.index(name)
            lst.lst_set_timed_site(k)
            site_ms[name] = round(sum(step(i, k, gh=g_ext.handle)[1] for i in range(2)) / 2, 4)
        lst.lst_set_timed_site(-1)
        ext["site_ms"] = site_ms
        log(f"bench: plain with extensions {ext}")

    # ---- end to end from pinned host memory: H2D, the chain, track candidates to the host
    e2e = None
    if "e2e" in forms:
        keys = ("x", "y", "z", "module", "sensor", "px", "py", "pz", "q", "hits4")
        pinned = [{k: pool[i][k].cpu().pin_memory() for k in keys} for i in range(len(pool))]

        def e2e_step(i):
            h = {k: v.to(dev, non_blocking=True) for k, v in pinned[i % len(pinned)].items()}
            st, ev = lst.lst_build_event(g.handle, h, ws, cap, stream)
            if st != lst.LST_OK:
                raise lst.LSTError(st, lst.lst_last_error())
            tc = lst.lst_get_track_candidates(ev)
            lst.lst_release_event(ev)
            return tc

        for i in range(max(args.warmup, 4)):
            e2e_step(i)
        torch.cuda.synchronize()
        lat, n_e2e = [], 32
        t0 = time.perf_counter()
        for i in range(n_e2e):
            s0 = time.perf_counter()
            e2e_step(4 + i)
            lat.append((time.perf_counter() - s0) * 1e3)
        el = time.perf_counter() - t0
        e2e = {"events_per_s": round(n_e2e / el, 3), "latency_ms": percentiles(lat), "events": n_e2e,
               "boundary": "pinned host hits+seeds -> H2D -> chain -> track candidates on the host"}
        del pinned
        log(f"bench: e2e {e2e}")

    # ---- open-loop trace: Poisson arrivals, pile-up U[50, 250], served vs plain FIFO on the same trace
    trace = None
    if args.trace > 0 and "trace" in forms:
        spool = [lst.upload_event(make_event("serve", i), dev) for i in range(args.pool)]
        rng = np.random.Generator(np.random.PCG64(4999))
        arrivals = np.cumsum(rng.exponential(1.0 / args.rate, args.trace))
        ids = rng.integers(0, len(spool), args.trace)
        smax = max(int(t["x"].numel()) for t in spool)
        sseed = max(int(t["px"].numel()) for t in spool)
        s_one = lst.lst_workspace_bytes(g.handle, smax, sseed)
        lat_s, rate_s = run_trace(lst, g, spool, n_streams, max_batch, int(s_one * (n_streams * max_batch + 2)),
                                  arrivals, ids)
        lat_p, rate_p = run_trace(lst, g, spool, 1, 1, int(s_one * 3), arrivals, ids)
        trace = {"rate_offered": args.rate, "requests": args.trace, "pileup": "U[50,250]",
                 "served": {"events_per_s": round(rate_s, 2), "latency_ms": percentiles(lat_s)},
                 "plain_fifo": {"events_per_s": round(rate_p, 2), "latency_ms": percentiles(lat_p)}}
        log(f"bench: trace {trace}")
        sweep = []
        for rate in [float(r) for r in args.sweep.split(",") if r.strip()]:
            n = int(min(args.trace, max(200, 2 * rate)))  # about two seconds of arrivals, at least 200
            arr = np.cumsum(rng.exponential(1.0 / rate, n))
            sid = rng.integers(0, len(spool), n)
            ls_, rs_ = run_trace(lst, g, spool, n_streams, max_batch,
                                 int(s_one * (n_streams * max_batch + 2)), arr, sid)
            lp_, rp_ = run_trace(lst, g, spool, 1, 1, int(s_one * 3), arr, sid)
            sweep.append({"rate_offered": rate, "requests": n,
                          "served": {"events_per_s": round(rs_, 2), **percentiles(ls_)},
                          "plain_fifo": {"events_per_s": round(rp_, 2), **percentiles(lp_)}})
            log(f"bench: sweep {sweep[-1]}")
        trace["sweep_latency_ms"] = sweep

    # ---- batched: captured plan over B slots (pile-up U[140, 250]), graph replays
    batched = None
    if args.batch > 0 and "batched" in forms:
        bhost = make_events([("batch", i) for i in range(args.batch)])   # 64 distinct events
        bpool = [lst.upload_event(e, dev) for e in bhost]
        chain_batched = []
        bmax = max(int(t["x"].numel()) for t in bpool)
        bseed = max(int(t["px"].numel()) for t in bpool)
        evs = [bpool[i % len(bpool)] for i in range(args.batch)]
        reps = max(4, n_served // args.batch)

        def time_plan():
            plan = lst.Plan(g, args.batch, bmax, bseed)  # captured with the geometry's launch shapes
            for i, r in enumerate(plan.run(evs)):
                if len(chain_batched) < args.batch:  # the first replay of the first plan
                    hev = bhost[i % len(bhost)]
                    chain_batched.append(chain_bytes(r.counts()[0], hev.n_hits, int((hev.module >= 0).sum()),
                                                     geom.n_modules, int(geom.map_targets.size), hev.n_seeds))
                r.close()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                for r in plan.run(evs):
                    r.close()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            plan.close()
            del plan
            return el

        el = time_plan()
        batched = {"events_per_s": round(reps * args.batch / el, 2), "events_per_launch": args.batch,
                   "ms_per_launch": round(el / reps * 1e3, 3), "pileup": "U[140,250]", "form": "hipGraph replay",
                   "launch_shapes": "tuned" if tuned else "default"}
        if tuned:
            g.set_launch_config({})
            el_d = time_plan()
            g.set_launch_config(tuned)
            batched["default_shapes_events_per_s"] = round(reps * args.batch / el_d, 2)
        bb = float(np.mean(chain_batched))
        batched["chain_bytes_per_event"] = int(bb)
        batched["chain_hbm_frac"] = round(batched["events_per_s"] * bb / (HBM_PEAK_GBS * 1e9), 5)
        log(f"bench: batched {batched}")

    # ---- device-to-device copy of a known size: achievable HBM bandwidth, and the reference
    # dispatch for scaling the FETCH_SIZE / WRITE_SIZE counters
    copy = None
    if "copy" in forms:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)  # an elementwise kernel: reads nbytes, writes nbytes
        torch.cuda.synchronize()
        reps = 10
        t0 = time.perf_counter()
        for _ in range(reps):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        copy = {"bytes_per_copy": nbytes, "kernel": "torch.mul(x, 1.0) over 2^28 float32",
                "read_plus_write_GBs": round(2 * nbytes * reps / el / 1e9, 1)}
        del src, dst
        log(f"bench: copy {copy}")

    # ---- vector-issue calibration: a kernel of 16 independent FMAs per round and nothing else, at
    # 8 waves per SIMD; its issue rate is the ceiling the counter summaries normalise against
    probe = None
    if "probe" in forms:
        n_blocks, iters = 4096, 4000
        out_p = torch.empty(n_blocks * 256, dtype=torch.float32, device=dev)
        lst.lst_probe_valu(n_blocks, 10, out_p)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        lst.lst_probe_valu(n_blocks, iters, out_p)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        insts = n_blocks * 4 * 16 * iters           # wave64 FMA instructions issued
        probe = {"kernel": "16 independent FMA chains per thread, 4096 x 256 threads, 4000 rounds",
                 "ms": round(ms, 4), "valu_insts": insts,
                 "insts_per_cu_per_clock_at_2.4GHz": round(insts / (ms * 1e-3 * 2.4e9 * 256), 4)}
        del out_p
        log(f"bench: probe {probe}")

    # ---- roofline of the dominant kernel: algorithmic bytes of the events of each batched launch
    # divided by that launch's HIP-event duration, summed over the served run's launches
    roof = None
    if launches and all(v[1] is not None for v in launches.values()):
        tot_b = sum(v[1] for v in launches.values())
        tot_s = sum(v[0] for v in launches.values()) / 1e3
        ach = tot_b / tot_s / 1e9
        tr = measured_traffic(sites[dom])
        ev_per_launch = n_served / len(launches)
        roof = {"bound": "hbm", "kernel": sites[dom], "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5),
                "traffic": None if tr is None else int(tr["hbm_bytes_per_event"] * ev_per_launch),
                "launches": len(launches), "bytes_per_launch": int(tot_b / len(launches)),
                "launch_ms": round(tot_s * 1e3 / len(launches), 4),
                "events_per_launch": round(ev_per_launch, 2),
                "traffic_source": None if tr is None else tr["profile"],
                # the kernel's VALU issue rate over the 2.0 per CU per clock of the FP32 peak, from
                # the same recorded counter run (it is issue-bound, not HBM-bound)
                "valu_issue_frac": None if tr is None else tr.get("valu_issue_frac"),
                "valu_issue_source": None if tr is None else tr.get("counters_profile")}
    out = {
        "metric": "events/s + p50/p99 event latency, PU200-like synthetic, served vs plain, 1 GPU",
        "value": round(value, 3), "unit": "events/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOAD[args.workload], "events_in_pool": args.pool,
                   "mean_hits": int(np.mean([e.n_hits for e in host])),
                   "mean_seeds": int(np.mean([e.n_seeds for e in host])),
                   "form": f"served: {n_streams} streams x batches of {max_batch}, all requests available",
                   "step": f"one server round: {round_events} events through the whole chain",
                   "events_timed": n_served,
                   "latency": "served p50/p99 of the Poisson trace (500 events/s, pile-up U[50, 250])"},
        "latency_ms": trace["served"]["latency_ms"] if trace else None,
        "saturation_latency_ms": percentiles(served_lat),
        "launch_shapes": tuned, "plain": plain, "plain_graph": plain_graph, "stub16": stub16, "extensions": ext, "displaced": displaced, "e2e": e2e, "trace": trace, "batched": batched, "copy": copy, "valu_probe": probe,
        "roofline": roof,
    }
    if chain_served:
        # the whole chain against HBM: algorithmic bytes of an event through every stage
        cb = float(np.mean(chain_served))
        out["chain_roofline"] = {
            "bound": "hbm", "bytes_per_event": int(cb), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "roofline_events_per_s": round(HBM_PEAK_GBS * 1e9 / cb, 1),
            "served_frac": round(value * cb / (HBM_PEAK_GBS * 1e9), 5),
            "batched_frac": batched["chain_hbm_frac"] if batched else None,
            "bytes": "hits 16 B read + 20 B bucketed per hit, plus each stage's inputs read once and outputs "
                     "written once (" + ", ".join(CHAIN_SITES) + ")"}
    if not args.no_physics:
        # efficiency, fake and duplicate rates of the HIP track candidates of every pool event,
        # against the generator's truth (outside every timed region)
        from lstgen.truth_metrics import pooled_metrics
        pairs, pairs_ext, n_ext_tc = [], [], 0
        for ev, d in zip(host, pool):
            r = lst.run_event(g, d)
            pairs.append((ev, r.track_candidates()))
            r.close()
            if ext is not None:
                r = lst.run_event(g_ext, d)
                ty, off, hits, na, _, _ = r.extended_track_candidates()
                pairs_ext.append((ev, (ty, off, hits)))
                n_ext_tc += int((na > 0).sum())
                r.close()
        m = pooled_metrics(pairs)
        rnd = lambda v: {k: rnd(x) for k, x in v.items()} if isinstance(v, dict) else (
            round(v, 5) if isinstance(v, float) else v)
        out["physics"] = {k: rnd(m[k]) for k in ("events", "n_tracks", "n_tc", "efficiency", "fake_rate",
                                            "duplicate_rate", "by_type")}
        out["physics"]["match"] = "a candidate matches a track when >= 75% of its hits are the track's"
        out["physics"]["denominator"] = "generated tracks with pT > 0.9 GeV and |eta| < 2.4"
        if pairs_ext:
            mx = pooled_metrics(pairs_ext)
            out["physics"]["extended"] = {"fraction_extended": round(n_ext_tc / max(1, mx["n_tc"]), 5),
                                          **{k: rnd(mx[k]) for k in ("efficiency", "fake_rate", "duplicate_rate")}}
        log(f"bench: physics {json.dumps(m)}")
    if not args.no_cpu:
        n_work = args.cpu_workers or min(16, len(os.sched_getaffinity(0)))
        rate, wall, per_event, steps = cpu_baseline(args.workload, host, n_work)
        model = "unknown CPU"
        try:
            with open("/proc/cpuinfo") as fh:
                model = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
        except (OSError, StopIteration):
            pass
        out["cpu_baseline"] = {"value": round(rate, 4), "unit": "events/s", "cores": n_work, "kind": "oracle",
                               "sample": f"{n_work} {args.workload} events (the first {min(n_work, len(host))} "
                                         f"of the pool, cycled), one per process, all at once: serial FP32 C "
                                         f"oracle, full chain, {wall:.1f} s wall; per event "
                                         f"{per_event[len(per_event) // 2]:.2f} s median; {model}",
                               "serial_stage_s": steps}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
