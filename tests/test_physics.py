"""Physics performance against generator truth (Section 3's hit-based matching), on the CPU.

The metric code is pinned on a hand-built event whose figures are counted by
hand; the oracle's track candidates on PU200-like events are then held to
the qualitative results the paper reports: high efficiency above the pT
turn-on, pT5 carrying most of it, pLS the largest fake share by type, and a
low duplicate rate after cross-cleaning.
"""
from types import SimpleNamespace

import numpy as np
import pytest

from lstgen.truth_metrics import match_candidates, pooled_metrics, tc_metrics


def _hand_event():
    # Tracks: 0 and 1 in the denominator; 2 below the pT threshold; 3 outside |eta| < 2.4.
    tracks = dict(pt=np.array([1.0, 2.0, 0.5, 3.0]), eta=np.array([0.0, 1.0, 0.0, 3.0]),
                  d0=np.array([0.0, -0.015, 0.0, 0.0]))
    sim = np.array([0, 0, 0, 0, 0, 0, 0,      # hits 0-6: track 0
                    1, 1, 1, 1,               # hits 7-10: track 1
                    2, 2,                     # hits 11-12: track 2
                    3, 3, 3, 3,               # hits 13-16: track 3
                    -1, -1, -1])              # hits 17-19: noise
    # Candidates (type codes: 0 pT5, 1 pT3, 2 T5, 3 pLS):
    tcs = [(0, [0, 1, 2, 3]),        # 4/4 of track 0           -> track 0
           (2, [4, 5, 6, 7]),        # 3/4 of track 0, exactly  -> track 0 (duplicate pair with the first)
           (1, [8, 9, 17, 18]),      # 2/4 of track 1           -> fake
           (3, [13, 14, 15, 16]),    # track 3, outside the denominator: matched, not counted for efficiency
           (2, [9, 10, 11, 12])]     # 2/4 of track 1, 2/4 of track 2 -> fake
    types = np.array([t for t, _ in tcs])
    off = np.concatenate([[0], np.cumsum([len(h) for _, h in tcs])])
    hits = np.concatenate([h for _, h in tcs])
    return SimpleNamespace(sim=sim, tracks=tracks), types, off, hits


def test_metrics_hand_counted():
    ev, types, off, hits = _hand_event()
    assert match_candidates(ev.sim, off, hits).tolist() == [0, 0, -1, 3, -1]
    m = tc_metrics(ev, types, off, hits)
    assert m["n_tc"] == 5 and m["n_tracks"] == 2
    assert m["efficiency"] == 0.5            # track 0 found, track 1 not
    assert m["fake_rate"] == 2 / 5
    assert m["duplicate_rate"] == 2 / 5      # both candidates of track 0
    bt = m["by_type"]
    assert bt["pT5"] == {"n": 1, "fake_rate": 0.0, "duplicate_rate": 1.0, "efficiency": 0.5}
    assert bt["T5"] == {"n": 2, "fake_rate": 0.5, "duplicate_rate": 0.5, "efficiency": 0.0}
    assert bt["pT3"] == {"n": 1, "fake_rate": 1.0, "duplicate_rate": 0.0, "efficiency": 0.0}
    assert bt["pLS"] == {"n": 1, "fake_rate": 0.0, "duplicate_rate": 0.0, "efficiency": 0.0}
    pt_bins = {(lo, hi): (n, e) for lo, hi, n, e in m["efficiency_vs_pt"]}
    assert pt_bins[(1.0, 1.5)] == (1, 1.0) and pt_bins[(2.0, 5.0)] == (1, 0.0)
    assert pt_bins[(0.8, 0.9)] == (0, None)  # track 2 (0.5 GeV) is below every bin
    d0_bins = {(lo, hi): (n, e) for lo, hi, n, e in m["efficiency_vs_d0"]}
    assert d0_bins[(0.0, 0.01)] == (1, 1.0) and d0_bins[(0.01, 0.02)] == (1, 0.0)
    # A stricter match turns the 3/4 candidate into a fake.
    m2 = tc_metrics(ev, types, off, hits, frac=0.8)
    assert m2["fake_rate"] == 3 / 5 and m2["duplicate_rate"] == 0.0


def test_pooling_keeps_events_apart():
    """Two copies of one event pool to the same rates, and no track of one is matched from the other."""
    ev, types, off, hits = _hand_event()
    one = tc_metrics(ev, types, off, hits)
    two = pooled_metrics([(ev, (types, off, hits))] * 2)
    assert two["n_tc"] == 10 and two["n_tracks"] == 4
    for k in ("efficiency", "fake_rate", "duplicate_rate"):
        assert two[k] == one[k]


@pytest.fixture(scope="module")
def oracle_pu200():
    from oracle_pool import oracle_many
    return oracle_many([("pu200_seeded", 1), ("pu200", 2)])


@pytest.mark.slow
def test_oracle_physics_pu200_seeded(oracle_pu200):
    ev, snap = oracle_pu200[0]
    m = tc_metrics(ev, *snap.tc())
    bt = m["by_type"]
    assert m["n_tracks"] > 7000
    assert m["efficiency"] > 0.93
    assert m["fake_rate"] < 0.12 and m["duplicate_rate"] < 0.02
    # pT5 carries most of the efficiency and is the cleanest type; pLS is the least pure.
    assert bt["pT5"]["efficiency"] > 0.8 and bt["pT5"]["efficiency"] == max(b["efficiency"] for b in bt.values())
    assert bt["pT5"]["fake_rate"] < 0.02
    assert bt["pLS"]["fake_rate"] == max(b["fake_rate"] for b in bt.values())
    for lo, hi, n, e in m["efficiency_vs_pt"]:
        if lo >= 1.0:
            assert n > 100 and e > 0.9, (lo, hi, n, e)


@pytest.mark.slow
def test_oracle_physics_pu200_unseeded(oracle_pu200):
    """Without pixel seeds every candidate is a T5: lower efficiency, no pixel types."""
    ev, snap = oracle_pu200[1]
    m = tc_metrics(ev, *snap.tc())
    bt = m["by_type"]
    assert bt["T5"]["n"] == m["n_tc"] and bt["pT5"]["n"] == bt["pT3"]["n"] == bt["pLS"]["n"] == 0
    assert 0.8 < m["efficiency"] < 0.95
    assert m["fake_rate"] < 0.15 and m["duplicate_rate"] < 0.01


@pytest.mark.slow
def test_oracle_extensions_pu200_seeded(oracle_pu200):
    """Track extensions (Section 2.5): a large share of the candidates is lengthened, mostly
    with the matched track's own hits, and the physics figures do not get worse."""
    ev, snap = oracle_pu200[0]
    ty, off, hits = snap.tc()
    na, t3, _, xo, xh = snap.extensions()
    frac = (na > 0).mean()
    assert 0.25 < frac < 0.6          # the paper: about half
    assert np.all(na[ty == 3] == 0) and np.all((na >= 0) & (na <= 2))
    assert np.array_equal(np.diff(xo) - np.diff(off), 2 * na)
    sim = np.asarray(ev.sim)
    m = match_candidates(sim, off, hits)
    ok = [np.all(sim[xh[xo[j] + off[j + 1] - off[j]:xo[j + 1]]] == m[j]) for j in np.nonzero((na > 0) & (m >= 0))[0]]
    assert np.mean(ok) > 0.9
    base, ext = tc_metrics(ev, ty, off, hits), tc_metrics(ev, ty, xo, xh)
    assert ext["efficiency"] >= base["efficiency"] - 0.002
    assert ext["fake_rate"] <= base["fake_rate"] + 0.002
    assert ext["duplicate_rate"] <= base["duplicate_rate"] + 0.002
