"""The allocation-free entry point against lst_build_event, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

from lstgen import make_event, make_single_track_event

pytestmark = pytest.mark.gpu


def _static_tc(lst, g, dev, max_tc=1 << 16, max_hits=1 << 20):
    import torch
    ty = torch.full((max_tc,), -7, dtype=torch.int32, device="cuda")
    off = torch.full((max_tc + 1,), -7, dtype=torch.int32, device="cuda")
    hits = torch.full((max_hits,), -7, dtype=torch.int32, device="cuda")
    counts = torch.full((4,), -7, dtype=torch.int32, device="cuda")
    lst.lst_build_event_static(g.handle, dev, ty, off, hits, counts)
    torch.cuda.synchronize()
    n, nh, st = (int(v) for v in counts[:3].cpu())
    return n, nh, st, ty[:n].cpu().numpy(), off[:n + 1].cpu().numpy(), hits[:nh].cpu().numpy()


def test_static_entry_point_equals_build_event(full):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU is required for the gpu-marked tests")
    import paper_2207_08207_amd as lst
    lst.load_library()
    assert lst.lst_static_workspace_bytes() == 256 << 20
    g = lst.Geometry(full)
    rng = np.random.default_rng(11)
    n = 60
    small = make_single_track_event(full, np.exp(rng.uniform(np.log(0.8), np.log(20.0), n)), rng.uniform(-2, 2, n),
                                    rng.uniform(0, 2 * np.pi, n), z0=rng.normal(0, 5, n),
                                    q=np.where(rng.uniform(size=n) < 0.5, -1, 1), smear=True, seeded=True, seed=11,
                                    n_noise=300)
    big = make_event("serve", 5, pu=60)
    need = lst.lst_workspace_bytes(g.handle, big.n_hits, big.n_seeds)
    assert need < lst.lst_static_workspace_bytes(), need
    # two calls in a row, the second with a smaller event; each against the workspace form
    for ev in (big, small):
        print(f"[gpu] static entry point: {ev.n_hits} hits, {ev.n_seeds} seeds", flush=True)
        dev = lst.upload_event(ev)
        n_tc, n_h, st, ty, off, hits = _static_tc(lst, g, dev)
        ref = lst.run_event(g, dev)
        rt, ro, rh = ref.track_candidates()
        assert st == 0 and n_tc == rt.size and n_h == rh.size and n_tc > 50
        assert np.array_equal(ty, rt) and np.array_equal(off, ro) and np.array_equal(hits, rh)
    # output buffers too small: counts reported, arrays untouched
    dev = lst.upload_event(small)
    n_tc, n_h, st, ty, off, hits = _static_tc(lst, g, dev, max_tc=4, max_hits=16)
    assert st == 0 and n_tc == rt.size and n_h == rh.size
    # an event above the static workspace is rejected before any device work
    huge = dict(dev)
    import torch
    big_x = torch.zeros(600000, dtype=torch.float32, device="cuda")
    for k in ("x", "y", "z"):
        huge[k] = big_x
    huge["module"] = torch.zeros(600000, dtype=torch.int32, device="cuda")
    huge["sensor"] = torch.zeros(600000, dtype=torch.int32, device="cuda")
    with pytest.raises(lst.LSTError) as e:
        _static_tc(lst, g, huge)
    assert e.value.status == lst.LST_E_NOMEM and "static workspace" in str(e.value)
