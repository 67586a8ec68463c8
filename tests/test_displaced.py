"""Displaced tracks (Section 3): the same chain with a wider impact-parameter bound.

* the generator's helix through a displaced vertex: the vertex lies on it
  with the drawn direction, and |d0| is the helix's closest approach to the
  beam line (brute force over the arc length);
* closed form: the exact hits of one helix with |d0| up to 3 cm give, with
  the bound at 3.6 cm, one MD per crossed module and one LS / T3 / T5 per
  chain of 2 / 3 / 5 map-linked MDs (every cut passes), and one T5 after
  duplicate removal; with the default 0.1 cm bound such tracks lose them;
* the displaced-muon sample: efficiency above 0.8 in every bin of the
  vertex's transverse displacement with the wide bound, and falling below
  0.5 beyond 1 cm with the default bound.
"""
import numpy as np
import pytest

import oracle
from lstgen import make_event, make_single_track_event
from lstgen.events import helix_from_vertex
from lstgen.geometry import K_CURV, helix_point
from lstgen.truth_metrics import pooled_metrics

from test_oracle_pins import _chain_counts, _tracks
from truth import md_surfaces

CUBE_BOUND = 3.6  # cm: above the largest transverse displacement of the 5 cm cube (3.54 cm)


def test_helix_through_vertex():
    rng = np.random.default_rng(5)
    n = 64
    v = rng.uniform(-2.5, 2.5, (3, n))
    psi = rng.uniform(0, 2 * np.pi, n)
    kap = rng.choice([-1, 1], n) * K_CURV / np.exp(rng.uniform(np.log(0.8), np.log(50), n))
    lam = np.sinh(rng.uniform(-2.4, 2.4, n))
    phi0, d0, z0, sv = helix_from_vertex(v[0], v[1], v[2], psi, kap, lam)
    x, y, z = helix_point(phi0, d0, z0, kap, lam, sv)
    assert np.allclose([x, y, z], v, atol=1e-9)
    x2, y2, _ = helix_point(phi0, d0, z0, kap, lam, sv + 1e-6)
    assert np.allclose(np.angle(np.exp(1j * (np.arctan2(y2 - y, x2 - x) - psi))), 0, atol=1e-6)
    s = np.linspace(-60, 60, 120001)
    for i in range(0, n, 8):
        xs, ys, _ = helix_point(phi0[i], d0[i], z0[i], kap[i], lam[i], s)
        assert abs(np.hypot(xs, ys).min() - abs(d0[i])) < 1e-6
    assert np.all(np.abs(d0) <= np.hypot(v[0], v[1]) + 1e-12)


@pytest.mark.parametrize("bound", [CUBE_BOUND, None])
def test_single_displaced_track_closed_form(bound, full):
    og = oracle.OracleGeometry(full, d0_max=bound)
    pt, eta, phi, z0, q = _tracks(40, 77, 2.4)
    d0 = np.random.default_rng(78).uniform(-3.0, 3.0, pt.size)
    n_eligible = n_lost = 0
    for i in range(pt.size):
        cr = md_surfaces(full, pt[i], eta[i], phi[i], z0[i], d0[i], q[i])
        ev = make_single_track_event(full, pt[i], eta[i], phi[i], z0=z0[i], d0=d0[i], q=q[i])
        r = oracle.run(og, ev, last=oracle.ST_T5)
        mds = [c[2] for c in cr if c[2] >= 0]
        chains = _chain_counts(full, mds)
        if bound is not None:
            assert r.count(oracle.ST_MD) == len(mds)
            assert r.count(oracle.ST_LS) == chains[2]
            assert r.count(oracle.ST_T3) == chains[3]
            assert r.count(oracle.ST_T5) == chains[5]
            _, keep, _ = r.stage(oracle.ST_T5)
            assert keep.sum() == (1 if chains[5] else 0)
            n_eligible += chains[5] > 0
        elif chains[5] and abs(d0[i]) > 1.0:
            n_eligible += 1
            n_lost += r.count(oracle.ST_T5) == 0
    if bound is not None:
        assert n_eligible >= 20
    else:
        assert n_eligible >= 10 and n_lost >= 0.8 * n_eligible


@pytest.mark.slow
def test_cube_efficiency_vs_displacement(full):
    ogs = {b: oracle.OracleGeometry(full, d0_max=b) for b in (None, CUBE_BOUND)}
    for b, og in ogs.items():
        pairs = []
        for k in range(20):
            ev = make_event("cube", k)
            pairs.append((ev, oracle.run(og, ev).tc()))
        m = pooled_metrics(pairs)
        bins = [(lo, n, e) for lo, hi, n, e in m["efficiency_vs_dxy"] if n >= 20]
        assert len(bins) >= 5
        if b is None:
            assert all(e < 0.5 for lo, n, e in bins if lo >= 1.0)
        else:
            assert all(e > 0.8 for lo, n, e in bins), bins
            assert m["fake_rate"] < 0.05 and m["duplicate_rate"] < 0.02
