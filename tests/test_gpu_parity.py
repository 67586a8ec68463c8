"""HIP library versus the CPU oracle, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import oracle
from lstgen import make_event, make_single_track_event
from lstgen.events import Event, make_tiny_event

from oracle_pool import oracle_many
from parity import compare_event, compare_tc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lst():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU is required for the gpu-marked tests")
    import paper_2207_08207_amd as lst
    lst.load_library()
    return lst


@pytest.fixture(scope="module")
def gbarrel(lst, barrel):
    return lst.Geometry(barrel)


@pytest.fixture(scope="module")
def gfull(lst, full):
    return lst.Geometry(full)


def _run(lst, g, ev, **kw):
    print(f"[gpu] {ev.name or 'event'}: {ev.n_hits} hits, {ev.n_seeds} seeds", flush=True)
    return lst.run_event(g, lst.upload_event(ev), **kw)


def test_module_windows_bit_exact(gbarrel, gfull, obarrel, ofull):
    for g, og in ((gbarrel, obarrel), (gfull, ofull)):
        a = g.module_constants()
        b = og.module_consts()
        assert a.dtype == b.dtype == np.float32
        assert np.array_equal(a.view(np.int32), b.view(np.int32))


@pytest.mark.parametrize("ev_no", range(10))
def test_parity_tiny(ev_no, lst, gbarrel, obarrel):
    ev = make_event("tiny", ev_no)
    r = _run(lst, gbarrel, ev)
    o = oracle.run(obarrel, ev)
    stats = compare_event(r, o, stages=range(4))
    compare_tc(r, o)
    assert stats["T5"]["oracle"] > 50


@pytest.mark.parametrize("seed", range(3))
def test_parity_tiny_seeded_ragged(seed, lst, gbarrel, obarrel, barrel):
    """Barrel tracks with pixel seeds, unsmeared and smeared, plus noise: every stage incl. pT3/pT5/TC."""
    rng = np.random.default_rng(seed)
    n = 37 + 11 * seed  # not a multiple of any block size
    ev = make_single_track_event(barrel, np.exp(rng.uniform(np.log(0.8), np.log(20.0), n)),
                                 rng.uniform(-0.5, 0.5, n), rng.uniform(0, 2 * np.pi, n), z0=rng.normal(0, 5, n),
                                 q=np.where(rng.uniform(size=n) < 0.5, -1, 1), smear=bool(seed % 2), seeded=True,
                                 seed=seed, n_noise=50)
    r = _run(lst, gbarrel, ev)
    o = oracle.run(obarrel, ev)
    compare_event(r, o)
    assert compare_tc(r, o) > 0


def test_parity_unsorted_module_map(lst, full):
    """A module map whose targets are not in increasing module order (each module's list
    reversed): the segment search finds partners linked module by linked module and must
    still report them in map order, as the oracle does."""
    import copy
    geom = copy.copy(full)
    mo, mt = full.map_offsets, full.map_targets.copy()
    for m in range(full.n_modules):
        mt[mo[m]:mo[m + 1]] = mt[mo[m]:mo[m + 1]][::-1].copy()
    geom.map_targets = mt
    assert any(mo[m + 1] - mo[m] > 1 for m in range(full.n_modules))
    ev = make_event("pu200_seeded", 2)
    r = _run(lst, lst.Geometry(geom), ev)
    o = oracle.run(oracle.OracleGeometry(geom), ev)
    stats = compare_event(r, o, stages=range(3))
    assert stats["LS"]["oracle"] > 100000
    compare_tc(r, o)


def test_parity_pu200_seeded_full_event(lst, gfull, ofull):
    """The full-size PU200-like event with pixel seeds, all stages, every object."""
    ev = make_event("pu200_seeded", 0)
    r = _run(lst, gfull, ev)
    o = oracle.run(ofull, ev)
    stats = compare_event(r, o)
    n = compare_tc(r, o)
    print("[gpu] pu200_seeded#0", stats, "TC", n, flush=True)
    assert stats["T5"]["oracle"] > 1000 and n > 1000


# Many full-size events: the oracle runs them in parallel processes once per module.
MANY = [("pu200_seeded", k) for k in range(1, 21)] + [("pu200", k) for k in range(2, 22)]
BATCH = [("batch", k) for k in range(8)]
PLAN64 = [("batch", k) for k in range(64)]      # the benchmark's 64-slot plan
SERVE = [("serve", k) for k in range(8)]        # pile-up U[50, 250], the serving workload


@pytest.fixture(scope="module")
def many_oracle():
    specs = MANY + [s for s in PLAN64 if s not in MANY] + SERVE
    print(f"[cpu] oracle on {len(specs)} full-size events in parallel", flush=True)
    return dict(zip(specs, oracle_many(specs)))


@pytest.mark.parametrize("spec", MANY, ids=[f"{c}-{k}" for c, k in MANY])
def test_parity_many_events(spec, lst, gfull, many_oracle):
    """Twenty seeded and twenty unseeded PU200-like events, every stage and the track candidates."""
    ev, o = many_oracle[spec]
    r = _run(lst, gfull, ev)
    compare_event(r, o)
    assert compare_tc(r, o) > 1000


def test_physics_metrics_from_hip_candidates(lst, gfull, many_oracle):
    """Efficiency, fake and duplicate rates of the HIP candidates equal the oracle's, pooled over events."""
    from lstgen.truth_metrics import pooled_metrics
    for config in ("pu200_seeded", "pu200"):
        specs = [s for s in MANY if s[0] == config][:8]
        hip, orc = [], []
        for s in specs:
            ev, o = many_oracle[s]
            r = _run(lst, gfull, ev)
            hip.append((ev, r.track_candidates()))
            orc.append((ev, o.tc()))
            r.close()
        mh, mo = pooled_metrics(hip), pooled_metrics(orc)
        print(f"[gpu] {config} x{len(specs)}: efficiency {mh['efficiency']:.4f} fake {mh['fake_rate']:.4f} "
              f"duplicate {mh['duplicate_rate']:.4f}", flush=True)
        assert mh == mo
        assert mh["efficiency"] > (0.93 if config == "pu200_seeded" else 0.8)


@pytest.fixture(scope="module")
def gfull_ext(lst, full):
    g = lst.Geometry(full)
    g.set_track_extensions(True)
    return g


def _compare_ext(r, o):
    """Extended collection, added-MD counts, triplet indices and fit attributes: all bit-exact."""
    tg, og_, hg, ng, t3g, ag = r.extended_track_candidates()
    na, t3, at, oo, ho = o.extensions()
    to, _, _ = o.tc()
    assert np.array_equal(tg, to), "types differ"
    assert np.array_equal(ng, na), "added-MD counts differ"
    assert np.array_equal(t3g, t3), "extension triplets differ"
    assert np.array_equal(og_, oo) and np.array_equal(hg, ho), "extended hit lists differ"
    assert np.array_equal(ag.view(np.int32), at.astype(np.float32).view(np.int32)), "extension attributes differ"
    return int((ng > 0).sum()), len(tg)


def test_extensions_equal_oracle(lst, gfull_ext, many_oracle):
    """Track extensions of seeded and unseeded PU200-like events against the oracle, the base
    candidates unchanged by the extra step."""
    n_ext = n_tc = 0
    for s in [x for x in MANY if x[0] == "pu200_seeded"][:6] + [x for x in MANY if x[0] == "pu200"][:3]:
        ev, o = many_oracle[s]
        r = _run(lst, gfull_ext, ev)
        compare_tc(r, o)
        a, b = _compare_ext(r, o)
        n_ext += a
        n_tc += b
        r.close()
    print(f"[gpu] extensions: {n_ext} of {n_tc} candidates extended", flush=True)
    assert 0.25 * n_tc < n_ext < 0.6 * n_tc


def test_extensions_small_and_empty_events(lst, barrel, obarrel):
    g = lst.Geometry(barrel)
    g.set_track_extensions(True)
    for seed in range(3):
        rng = np.random.default_rng(100 + seed)
        n = 23 + 17 * seed
        ev = make_single_track_event(barrel, np.exp(rng.uniform(np.log(0.8), np.log(20.0), n)),
                                     rng.uniform(-0.5, 0.5, n), rng.uniform(0, 2 * np.pi, n), z0=rng.normal(0, 5, n),
                                     q=np.where(rng.uniform(size=n) < 0.5, -1, 1), smear=bool(seed % 2),
                                     seeded=seed != 1, seed=seed, n_noise=30)
        r = _run(lst, g, ev)
        _compare_ext(r, oracle.run(obarrel, ev))
        r.close()
    empty = Event(x=np.zeros(0, np.float32), y=np.zeros(0, np.float32), z=np.zeros(0, np.float32),
                  module=np.zeros(0, np.int32), sensor=np.zeros(0, np.int32), sim=np.zeros(0, np.int32))
    r = _run(lst, g, empty)
    ty, off, hits, na, t3, at = r.extended_track_candidates()
    assert len(ty) == 0 and list(off) == [0] and len(hits) == 0
    r.close()


def test_extensions_disabled_is_an_error(lst, gbarrel):
    ev = make_event("tiny", 0)
    r = _run(lst, gbarrel, ev)
    with pytest.raises(lst.LSTError) as ei:
        r.extended_track_candidates()
    assert ei.value.status == lst.LST_E_STATE
    r.close()
    lib = lst.load_library()
    assert lib.lst_set_track_extensions(gbarrel.handle, 2) == lst.LST_E_INVALID
    assert lib.lst_set_track_extensions(None, 1) == lst.LST_E_INVALID


def test_extensions_in_captured_plan(lst, gfull_ext, many_oracle):
    """The extension step inside a captured batch plan, event by event against the oracle."""
    evs = [many_oracle[s][0] for s in BATCH[:4]]
    dev = [lst.upload_event(e) for e in evs]
    plan = lst.Plan(gfull_ext, len(evs), max(e.n_hits for e in evs), max(e.n_seeds for e in evs))
    for _ in range(2):  # two replays
        for r, s in zip(plan.run(dev), BATCH[:4]):
            _compare_ext(r, many_oracle[s][1])
            r.close()
    plan.close()


def test_displaced_bound_windows_and_cube_events(lst, full, barrel, obarrel):
    """The displaced configuration (impact-parameter bound 3.6 cm): module windows and every stage
    of displaced-muon events bit-exact; the barrel with a 1 cm bound on small events."""
    g = lst.Geometry(full)
    g.set_impact_bound(3.6)
    og = oracle.OracleGeometry(full, d0_max=3.6)
    assert np.array_equal(g.module_constants().view(np.int32), og.module_consts().view(np.int32))
    n_t5 = 0
    for k in range(12):
        ev = make_event("cube", k)
        r = _run(lst, g, ev)
        o = oracle.run(og, ev)
        stats = compare_event(r, o)
        compare_tc(r, o)
        n_t5 += stats["T5"]["oracle"]
        r.close()
    assert n_t5 > 300
    gb = lst.Geometry(barrel)
    gb.set_impact_bound(1.0)
    ogb = oracle.OracleGeometry(barrel, d0_max=1.0)
    for k in range(3):
        ev = make_event("tiny", k)
        r = _run(lst, gb, ev)
        compare_event(r, oracle.run(ogb, ev), stages=range(4))
        r.close()
    lib = lst.load_library()
    for bad in (0.0, -1.0, 10.5, float("nan")):
        assert lib.lst_set_impact_bound(g.handle, bad) == lst.LST_E_INVALID


def test_parity_batch_plan_events(lst, gfull, many_oracle):
    """Eight pile-up U[140, 250] events in one captured plan, each against the oracle."""
    evs = [many_oracle[s][0] for s in BATCH]
    dev = [lst.upload_event(e) for e in evs]
    print(f"[gpu] plan of {len(evs)} batch events: hits {[e.n_hits for e in evs]}", flush=True)
    plan = lst.Plan(gfull, len(evs), max(e.n_hits for e in evs), max(e.n_seeds for e in evs))
    for r, s in zip(plan.run(dev), BATCH):
        o = many_oracle[s][1]
        compare_event(r, o)
        compare_tc(r, o)
        r.close()
    plan.close()


def test_parity_batch_plan_64_slots(lst, full, many_oracle):
    """The benchmark's batched form: 64 pile-up U[140, 250] events in one captured plan with the
    packaged MI355X launch shapes, every event against the oracle, on two replays."""
    import os
    g = lst.Geometry(full)
    shapes = os.path.join(os.path.dirname(lst.__file__), "launch_shapes_mi355x.json")
    g.load_launch_config(shapes)
    evs = [many_oracle[s][0] for s in PLAN64]
    dev = [lst.upload_event(e) for e in evs]
    print(f"[gpu] plan of 64 batch events: hits {min(e.n_hits for e in evs)}..{max(e.n_hits for e in evs)}",
          flush=True)
    plan = lst.Plan(g, len(evs), max(e.n_hits for e in evs), max(e.n_seeds for e in evs))
    for rep in range(2):
        for r, s in zip(plan.run(dev), PLAN64):
            o = many_oracle[s][1]
            compare_event(r, o)
            compare_tc(r, o)
            r.close()
    plan.close()


@pytest.mark.parametrize("spec", SERVE, ids=[f"{c}-{k}" for c, k in SERVE])
def test_parity_serve_events(spec, lst, gfull, many_oracle):
    """The serving workload's events (pile-up U[50, 250]) on the default geometry, every stage."""
    ev, o = many_oracle[spec]
    r = _run(lst, gfull, ev)
    compare_event(r, o)
    assert compare_tc(r, o) > 100


def test_parity_dense_seed_search(lst, gbarrel, obarrel, barrel):
    """Dense seeded fixtures: seeds with 256-1,024 and more than 1,024 passing triplets and with more
    than 16 pT5, i.e. the seed search's re-search past its per-seed caches and its ordered scan past
    the LDS list, object by object against the oracle."""
    from dense import dense_event, spread_event
    for ev in (dense_event(barrel), spread_event(barrel)):
        r = _run(lst, gbarrel, ev)
        o = oracle.run(obarrel, ev)
        compare_event(r, o)
        compare_tc(r, o)
        t3, _, _ = r.stage(oracle.ST_PT3)
        t5, _, _ = r.stage(oracle.ST_PT5)
        n3 = np.bincount(t3[:, 0], minlength=ev.n_seeds)
        n5 = np.bincount(t5[:, 0], minlength=ev.n_seeds)
        print(f"[gpu] {ev.name}: pT3 per seed {n3.tolist()}, pT5 per seed {n5.tolist()}", flush=True)
        if ev.name == "dense":
            assert n3.max() > 1024 and ((n3 > 256) & (n3 <= 1024)).any()
        else:
            assert n5.max() > 16 and n3.max() > 1024
        r.close()


def test_parity_pu200_unseeded(lst, gfull, ofull):
    ev = make_event("pu200", 1)
    r = _run(lst, gfull, ev)
    o = oracle.run(ofull, ev)
    compare_event(r, o, stages=range(4))
    compare_tc(r, o)


def test_empty_and_degenerate_events(lst, gbarrel, obarrel, barrel):
    empty = Event(x=np.zeros(0, np.float32), y=np.zeros(0, np.float32), z=np.zeros(0, np.float32),
                  module=np.zeros(0, np.int32), sensor=np.zeros(0, np.int32), sim=np.zeros(0, np.int32))
    r = _run(lst, gbarrel, empty)
    ty, off, hits = r.track_candidates()
    assert ty.size == 0 and list(off) == [0] and hits.size == 0
    # one track, unseeded; one bare seed; noise only
    for ev in (make_single_track_event(barrel, 2.0, 0.2, 1.0),
               make_single_track_event(barrel, 2.0, 0.2, 1.0, seeded=True),
               make_tiny_event(0, n_tracks=0, n_noise=300)):
        r = _run(lst, gbarrel, ev)
        o = oracle.run(obarrel, ev)
        compare_event(r, o)
        compare_tc(r, o)


def test_invalid_input_rejected(lst, gbarrel, barrel):
    ev = make_single_track_event(barrel, 2.0, 0.2, 1.0)
    bad = Event(x=ev.x, y=ev.y, z=ev.z, module=ev.module.copy(), sensor=ev.sensor, sim=ev.sim)
    bad.module[0] = barrel.n_modules + 5
    with pytest.raises(lst.LSTError) as e:
        _run(lst, gbarrel, bad)
    assert e.value.status == lst.LST_E_INVALID
    bad2 = Event(x=ev.x.copy(), y=ev.y, z=ev.z, module=ev.module, sensor=ev.sensor, sim=ev.sim)
    bad2.x[1] = np.nan
    with pytest.raises(lst.LSTError):
        _run(lst, gbarrel, bad2)
    # more hits than the device scans hold: rejected before any work is enqueued
    import ctypes
    import torch
    d = lst._event_desc(lst.upload_event(ev))
    d.n_hits = 8_000_001
    h = ctypes.c_void_p()
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    st = lst.load_library().lst_build_event(gbarrel.handle, ctypes.byref(d), None, lst._ptr(ws), int(ws.numel()),
                                            None, ctypes.byref(h))
    assert st == lst.LST_E_INVALID and not h.value


def test_capacity_overflow_reports_and_recovers(lst, gbarrel, obarrel):
    ev = make_event("tiny", 2)
    cap = lst.lst_default_capacity(ev.n_hits, ev.n_seeds)
    cap.ls = 100  # far below the ~500 segments of the event
    dev = lst.upload_event(ev)
    ws = lst.alloc_workspace(gbarrel, ev.n_hits, ev.n_seeds, cap)
    st, h = lst.lst_build_event(gbarrel.handle, dev, ws, cap)
    assert st == lst.LST_E_CAPACITY
    counts, req = lst.lst_get_stage_counts(h)
    assert counts[1] == 100 and req[1] > 100
    lst.lst_release_event(h)
    r = lst.run_event(gbarrel, dev, cap=cap)  # grows and reruns
    compare_tc(r, oracle.run(obarrel, ev))


def test_deterministic_repeats(lst, gfull):
    ev = make_event("pu200_seeded", 2)
    dev = lst.upload_event(ev)
    ref = None
    for _ in range(3):
        r = lst.run_event(gfull, dev)
        out = [r.stage(s) for s in range(7)] + [r.track_candidates()]
        flat = [a.tobytes() for tup in out for a in tup]
        if ref is None:
            ref = flat
        assert flat == ref


# ------------------------------------------------------------------ batches
def _tc_tuple(r):
    return tuple(a.tobytes() for a in r.track_candidates())


def test_batch_ragged_equals_oracle(lst, gbarrel, obarrel, barrel):
    """Events of different sizes (incl. an empty one) in one batched launch sequence."""
    evs = [make_event("tiny", k) for k in range(3)]
    evs.append(make_tiny_event(11, n_tracks=3, n_noise=7))
    rng = np.random.default_rng(5)
    n = 23
    evs.append(make_single_track_event(barrel, np.exp(rng.uniform(0, 2, n)), rng.uniform(-0.5, 0.5, n),
                                       rng.uniform(0, 6.28, n), z0=rng.normal(0, 5, n), q=1, smear=True,
                                       seeded=True, seed=5, n_noise=31))
    evs.append(Event(x=np.zeros(0, np.float32), y=np.zeros(0, np.float32), z=np.zeros(0, np.float32),
                     module=np.zeros(0, np.int32), sensor=np.zeros(0, np.int32), sim=np.zeros(0, np.int32)))
    print(f"[gpu] batch of {len(evs)} events: hits {[e.n_hits for e in evs]}", flush=True)
    res = lst.run_batch(gbarrel, [lst.upload_event(e) for e in evs])
    for ev, r in zip(evs, res):
        o = oracle.run(obarrel, ev)
        compare_event(r, o)
        compare_tc(r, o)


def test_batch_pu200_equals_plain(lst, gfull):
    evs = [make_event("pu200_seeded", k) for k in (3, 4, 5)]
    dev = [lst.upload_event(e) for e in evs]
    print("[gpu] batch of 3 pu200_seeded", flush=True)
    plain = [_tc_tuple(lst.run_event(gfull, d)) for d in dev]
    res = lst.run_batch(gfull, dev)
    assert [_tc_tuple(r) for r in res] == plain


def test_plan_replays_equal_eager(lst, gbarrel, obarrel):
    """A captured plan replayed several times, eager work in between, every replay checked."""
    evs = [make_event("tiny", k) for k in range(6)]
    dev = [lst.upload_event(e) for e in evs]
    eager = [_tc_tuple(lst.run_event(gbarrel, d)) for d in dev]
    plan = lst.Plan(gbarrel, 4, max(e.n_hits for e in evs), 0)
    for rep, sel in enumerate([[0, 1, 2, 3], [4, 5], [2, 0, 5, 1], [3]]):
        print(f"[gpu] plan replay {rep}: events {sel}", flush=True)
        res = plan.run([dev[k] for k in sel])
        assert [_tc_tuple(r) for r in res] == [eager[k] for k in sel]
        # the previous run's events must be released before the next run
        if rep == 0:
            st, _ = lst.lst_plan_run(plan.handle, [dev[0]], plan.stream)
            assert st == lst.LST_E_STATE
        for r in res:
            r.close()
        lst.run_event(gbarrel, dev[rep])  # eager work between replays
    r = plan.run([dev[1]])[0]
    o = oracle.run(obarrel, evs[1])
    compare_event(r, o, stages=range(4))
    compare_tc(r, o)


# ------------------------------------------------------------------ serving
def test_served_mix_equals_alone(lst, gfull):
    """Each result is the same alone (plain path) and in the served mix (continuous batching)."""
    evs = [make_event("serve", k) for k in range(6)]
    print("[gpu] serve events PU", [round(e.tracks["pu"]) for e in evs], flush=True)
    dev = [lst.upload_event(e) for e in evs]
    alone = [_tc_tuple(lst.run_event(gfull, d)) for d in dev]
    one = max(lst.lst_workspace_bytes(gfull.handle, e.n_hits, e.n_seeds) for e in evs)
    for n_streams, max_batch, pool, stagger in ((3, 4, 12 * one, 0.0), (2, 3, 2.2 * one, 0.002), (1, 1, 1.2 * one, 0.0)):
        print(f"[gpu] server streams={n_streams} batch={max_batch} pool={pool / 2**30:.2f} GiB", flush=True)
        srv = lst.Server(gfull, n_streams, max_batch, pool)
        t0 = srv.now()
        order = [3, 0, 5, 1, 4, 2, 0, 3]
        for i, k in enumerate(order):
            srv.submit(dev[k], i, t0 + stagger * i)
        got = {}

        def take(r):
            assert r["status"] == lst.LST_OK, r
            res = lst.EventResult(r["event"], None, lst.LST_OK)
            got[r["id"]] = _tc_tuple(res)
            assert r["done_s"] >= r["admit_s"] >= r["arrival_s"] - 1e-6
            res.close()

        srv.drain(len(order), take)
        srv.close()
        assert [got[i] for i in range(len(order))] == [alone[k] for k in order]


def test_server_reruns_capacity_overflow(lst, gfull):
    """A request whose first capacities are far too small is run again by the server with grown
    capacities; its result equals the plain path's, and the requests batched with it are unaffected."""
    evs = [make_event("serve", k) for k in (1, 2, 3)]
    dev = [lst.upload_event(e) for e in evs]
    alone = [_tc_tuple(lst.run_event(gfull, d)) for d in dev]
    one = max(lst.lst_workspace_bytes(gfull.handle, e.n_hits, e.n_seeds) for e in evs)
    srv = lst.Server(gfull, 2, 3, 6 * one)
    small = lst.lst_default_capacity(evs[1].n_hits, evs[1].n_seeds)
    small.ls, small.t3 = 1000, 1000          # far below the event's segments and triplets
    t0 = srv.now()
    srv.submit(dev[0], 0, t0)
    srv.submit(dev[1], 1, t0, cap=small)
    srv.submit(dev[2], 2, t0)
    got = {}

    def take(r):
        assert r["status"] == lst.LST_OK, r
        res = lst.EventResult(r["event"], None, lst.LST_OK)
        got[r["id"]] = _tc_tuple(res)
        res.close()

    srv.drain(3, take)
    assert srv.reruns() >= 1
    srv.close()
    assert [got[i] for i in range(3)] == alone


def test_server_with_extensions_and_displaced_bound(lst, full, gfull_ext, many_oracle):
    """The serving loop on a geometry with the extension step, and on one with the displaced
    bound: every result equal to the oracle's."""
    specs = [s for s in MANY if s[0] == "pu200_seeded"][:4]
    dev = [lst.upload_event(many_oracle[s][0]) for s in specs]
    one = max(lst.lst_workspace_bytes(gfull_ext.handle, many_oracle[s][0].n_hits, many_oracle[s][0].n_seeds)
              for s in specs)
    srv = lst.Server(gfull_ext, 2, 2, 5 * one)
    t0 = srv.now()
    for i, d in enumerate(dev):
        srv.submit(d, i, t0)
    seen = set()

    def take(r):
        assert r["status"] == lst.LST_OK, r
        res = lst.EventResult(r["event"], None, lst.LST_OK)
        _compare_ext(res, many_oracle[specs[r["id"]]][1])
        seen.add(r["id"])
        res.close()

    srv.drain(len(dev), take)
    srv.close()
    assert seen == set(range(len(dev)))

    g = lst.Geometry(full)
    g.set_impact_bound(3.6)
    og = oracle.OracleGeometry(full, d0_max=3.6)
    cube = [make_event("cube", k) for k in range(20, 26)]
    cdev = [lst.upload_event(e) for e in cube]
    one = max(lst.lst_workspace_bytes(g.handle, e.n_hits, e.n_seeds) for e in cube)
    srv = lst.Server(g, 2, 3, 7 * one)
    t0 = srv.now()
    for i, d in enumerate(cdev):
        srv.submit(d, i, t0)
    got = {}

    def take_c(r):
        assert r["status"] == lst.LST_OK, r
        res = lst.EventResult(r["event"], None, lst.LST_OK)
        got[r["id"]] = res.track_candidates()
        res.close()

    srv.drain(len(cdev), take_c)
    srv.close()
    for i, e in enumerate(cube):
        to, oo, ho = oracle.run(og, e).tc()
        tg, og_, hg = got[i]
        assert np.array_equal(tg, to) and np.array_equal(og_, oo) and np.array_equal(hg, ho)


def test_half_stubs_equal_oracle(lst, full, barrel):
    """MD stubs in binary16: every stage and the candidates bit-exact with the oracle's binary16 column."""
    g = lst.Geometry(full)
    g.set_stub_precision(16)
    og = oracle.OracleGeometry(full, stub16=True)
    ev = make_event("pu200_seeded", 5)
    r = _run(lst, g, ev)
    o = oracle.run(og, ev)
    stats = compare_event(r, o)
    compare_tc(r, o)
    r.close()
    assert stats["LS"]["oracle"] > 100000
    gb = lst.Geometry(barrel)
    gb.set_stub_precision(16)
    ogb = oracle.OracleGeometry(barrel, stub16=True)
    for k in range(3):
        ev = make_event("tiny", 10 + k)
        r = _run(lst, gb, ev)
        o = oracle.run(ogb, ev)
        compare_event(r, o, stages=range(4))
        compare_tc(r, o)
        r.close()
    lib = lst.load_library()
    assert lib.lst_set_stub_precision(gb.handle, 8) == lst.LST_E_INVALID
