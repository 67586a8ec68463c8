"""Launch shapes and the autotuner, through the C ABI (needs an MI355X)."""
import pytest

import oracle
from lstgen import make_event

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


def test_launch_shapes_do_not_change_results(lst, barrel, obarrel):
    """Every tunable site at 64 and at 128 threads per block gives the oracle's objects."""
    g = lst.Geometry(barrel)
    cfg = g.launch_config()
    assert cfg and set(cfg.values()) == {256}
    evs = [make_event("tiny", k) for k in (3, 4)]
    dev = [lst.upload_event(e) for e in evs]
    for block in (64, 128):
        print(f"[gpu] all tunable sites at {block} threads", flush=True)
        g.set_launch_config({n: block for n in cfg})
        assert set(g.launch_config().values()) == {block}
        for ev, d in zip(evs, dev):
            r = lst.run_event(g, d)
            o = oracle.run(obarrel, ev)
            compare_event(r, o)
            compare_tc(r, o)
    g.set_launch_config({})
    assert set(g.launch_config().values()) == {256}
    with pytest.raises(lst.LSTError):
        g.set_launch_config({"hits_count": 64})  # a fixed-shape site
    with pytest.raises(lst.LSTError):
        g.set_launch_config({"ls_count": 96})


def test_autotune_keeps_results(lst, full, ofull, tmp_path):
    g = lst.Geometry(full)
    evs = [make_event("pu200_seeded", k) for k in (7, 8)]
    dev = [lst.upload_event(e) for e in evs]
    print("[gpu] autotune on 2 pu200_seeded events", flush=True)
    res = g.autotune(dev, reps=1)
    assert res and all(b in (64, 128, 256) and ms > 0 for b, ms in res.values())
    print("[gpu] tuned", {k: v[0] for k, v in res.items()}, flush=True)
    path = tmp_path / "launch.json"
    g.save_launch_config(path)
    g2 = lst.Geometry(full)
    g2.load_launch_config(path)
    assert g2.launch_config() == g.launch_config()
    r = lst.run_event(g2, dev[0])
    o = oracle.run(ofull, evs[0])
    compare_event(r, o)
    compare_tc(r, o)


def test_tile_choices_do_not_change_results(lst, full, ofull):
    """Every tile at its extremes and at the autotuner's candidates gives the oracle's objects; the
    smallest values force every fallback path: no cached partners (every fill searches again), a
    one-entry seed list (the ordered scan of all objects), a one-bin slice table (bin by bin)."""
    g = lst.Geometry(full)
    g.set_track_extensions(True)
    base = g.tile_config()
    assert base == {"md_cache": 32, "ls_cache": 32, "t3_cache": 2, "t5_cache": 2, "pt3_cache": 256,
                    "pt5_cache": 16, "pass_list": 1024, "max_slices": 512, "ext_per_wave": 8, "ls_group": 0}
    ev = make_event("pu200_seeded", 9)
    print(f"[cpu] oracle on {ev.n_hits} hits", flush=True)
    o = oracle.run(ofull, ev)
    d = lst.upload_event(ev)
    configs = [dict(md_cache=0, ls_cache=0, t3_cache=0, t5_cache=0, pt3_cache=0, pt5_cache=0, pass_list=1,
                    max_slices=1, ext_per_wave=4, ls_group=1),
               dict(md_cache=1, ls_cache=1, t3_cache=1, t5_cache=1, pt3_cache=1, pt5_cache=1, pass_list=2,
                    max_slices=2, ext_per_wave=16, ls_group=16),
               dict(md_cache=16, ls_cache=8, pt3_cache=64, pt5_cache=4, pass_list=256, max_slices=128, ls_group=3),
               dict(ls_cache=4, pt3_cache=128, pt5_cache=8)]
    for cfg in configs:
        g.set_tile_config(base)
        g.set_tile_config(cfg)
        print(f"[gpu] tiles {g.tile_config()}", flush=True)
        r = lst.run_event(g, d)
        compare_event(r, o)
        compare_tc(r, o)
        na, t3, at, oo, ho = o.extensions()
        tg, og_, hg, ng, t3g, ag = r.extended_track_candidates()
        assert (og_ == oo).all() and (hg == ho).all() and (ng == na).all() and (t3g == t3).all()
        r.close()
    bad = dict(base)
    bad["ext_per_wave"] = 5
    with pytest.raises(lst.LSTError):
        g.set_tile_config(bad)
    with pytest.raises(lst.LSTError):
        g.set_tile_config({"pt3_cache": 257})
    assert g.tile_config()["pt3_cache"] != 257


def test_autotune_tiles_keeps_results(lst, full, ofull, tmp_path):
    g = lst.Geometry(full)
    evs = [make_event("pu200_seeded", k) for k in (10, 11)]
    dev = [lst.upload_event(e) for e in evs]
    print("[gpu] tile autotune on 2 pu200_seeded events", flush=True)
    res = g.autotune_tiles(dev, reps=1)
    print("[gpu] tiles", res, flush=True)
    assert set(res) == {n for n, _, _ in lst.lst_tiles()} - {"ext_per_wave"}
    assert all(ms > 0 for _, ms in res.values())
    path = tmp_path / "launch.json"
    g.save_launch_config(path)
    g2 = lst.Geometry(full)
    g2.load_launch_config(path)
    assert g2.tile_config() == g.tile_config()
    r = lst.run_event(g2, dev[0])
    o = oracle.run(ofull, evs[0])
    compare_event(r, o)
    compare_tc(r, o)
