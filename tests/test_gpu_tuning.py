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
