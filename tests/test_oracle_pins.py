"""Pins of the CPU oracle to facts that do not come from the oracle itself.

* closed form: exact hits of a helix above threshold give one MD per crossed
  module, one LS / T3 / T5 per chain of 2 / 3 / 5 of the track's MDs linked
  by the module map, and one T5 after duplicate removal; the
  fitted curvatures equal -q K / pT; the r-z and x-y chi2 vanish; the segment
  angles equal asin(kappa r / 2) at the other end;
* threshold: exact hits below the pT threshold give no MD where the
  curvature term dominates the window;
* library routine: the quintuplet circle fit equals numpy's least squares;
* brute force: the staged loops equal the closure over all combinations;
* invariance: relabelling hits does not change the track candidates;
* hand-derived cleaning outcomes for small fixtures (Section 2.5).
"""
import math

import numpy as np
import pytest

import oracle
from lstgen import make_event, make_single_track_event
from lstgen.events import Event, make_tiny_event
from lstgen.geometry import K_CURV, PT_MIN, surface_crossing

from truth import kappa_true, md_runs, md_surfaces

KMAX = K_CURV / PT_MIN


def _tracks(n, seed, eta_max, pt_lo=0.8, pt_hi=50.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    pt = np.exp(rng.uniform(math.log(pt_lo), math.log(pt_hi), n))
    eta = rng.uniform(-eta_max, eta_max, n)
    phi = rng.uniform(0, 2 * math.pi, n)
    z0 = rng.uniform(-15.0, 15.0, n)
    q = np.where(rng.uniform(0, 1, n) < 0.5, -1, 1)
    return pt, eta, phi, z0, q


# ------------------------------------------------------------------ geometry
def test_module_counts(barrel, full):
    assert barrel.n_modules == 5736
    assert full.n_modules == 19262
    for g in (barrel, full):
        off = g.map_offsets
        assert off[0] == 0 and off[-1] == g.map_targets.size
        assert np.all(np.diff(off) >= 0)
        assert g.map_targets.min() >= 0 and g.map_targets.max() < g.n_modules
        for m in range(0, g.n_modules, 97):
            row = g.map_targets[off[m]:off[m + 1]]
            assert np.all(np.diff(row) > 0)  # sorted, unique


def test_helix_crossings_lie_on_surfaces(full):
    pt, eta, phi, z0, q = _tracks(2000, 11, 2.4)
    kap = -q * K_CURV / pt
    lam = np.sinh(eta)
    d0 = np.full(pt.size, 0.03)
    for surf in full.surfaces():
        kind, _i, _s, _sen, pos = surf
        s, mod, x, y, z = surface_crossing(full, surf, phi, d0, z0, kap, lam)
        ok = mod >= 0
        if kind == "b":
            assert np.all(np.abs(np.hypot(x[ok], y[ok]) - pos) < 1e-9)
        else:
            assert np.all(np.abs(z[ok] - pos) < 1e-9)
        # on the helix: distance to the circle centre equals the radius
        cx = d0 * -np.sin(phi) - np.sin(phi) / kap
        cy = d0 * np.cos(phi) + np.cos(phi) / kap
        rr = np.hypot(x - cx, y - cy)
        assert np.all(np.abs(rr[ok] - 1.0 / np.abs(kap[ok])) < 1e-7 / np.abs(kap[ok]))
        assert np.all(np.abs(z[ok] - (z0[ok] + lam[ok] * s[ok])) < 1e-9)


def test_smear_within_pitch(barrel):
    from lstgen.events import _track_hits
    from lstgen.geometry import PITCH
    pt, eta, phi, z0, q = _tracks(200, 5, 0.5)
    kap = -q * K_CURV / pt
    lam = np.sinh(eta)
    d0 = np.zeros(pt.size)
    a = _track_hits(barrel, phi, d0, z0, kap, lam, False, np.random.Generator(np.random.PCG64(1)))
    b = _track_hits(barrel, phi, d0, z0, kap, lam, True, np.random.Generator(np.random.PCG64(1)))
    assert np.array_equal(a["module"], b["module"])
    ty = barrel.type[a["module"]]
    prphi = np.where(ty == 0, PITCH[0][0], PITCH[1][0])
    plong = np.where(ty == 0, PITCH[0][1], PITCH[1][1])
    ra = np.hypot(a["x"], a["y"])
    dphi = np.angle((b["x"] + 1j * b["y"]) / (a["x"] + 1j * a["y"]))
    assert np.all(np.abs(dphi * ra) <= prphi / 2 * (1 + 1e-9))
    assert np.all(np.abs(b["z"] - a["z"]) <= plong / 2 * (1 + 1e-9))
    assert np.all(np.abs(np.hypot(b["x"], b["y"]) - ra) < 1e-9)


def _crossing_table(geom, pt, eta, phi, z0, d0, q):
    kap = -q * K_CURV / pt
    lam = np.sinh(eta)
    per = {}
    for surf in geom.surfaces():
        kind, idx, side, sensor, _pos = surf
        s, mod, *_ = surface_crossing(geom, surf, phi, d0, z0, kap, lam)
        rec = per.setdefault((kind, idx, side), [None, None, None])
        if sensor == 0:
            rec[0], rec[1] = s, mod
        else:
            rec[2] = mod
    return per


@pytest.mark.parametrize("which", ["barrel", "full"])
def test_module_map_complete_on_truth(which, barrel, full):
    """Section 2.2: every pair of MDs of a track above threshold on consecutive surfaces is a map edge."""
    geom = barrel if which == "barrel" else full
    pt, eta, phi, z0, q = _tracks(6000, 21, 0.5 if which == "barrel" else 2.4)
    z0 = np.clip(z0 * 1.3, -19.9, 19.9)
    d0 = np.random.Generator(np.random.PCG64(3)).uniform(-0.1, 0.1, pt.size)
    per = _crossing_table(geom, pt, eta, phi, z0, d0, q)
    keys = list(per)
    S = np.stack([np.where(np.isfinite(per[k][0]), per[k][0], np.inf) for k in keys], 1)
    LO = np.stack([per[k][1] for k in keys], 1)
    UP = np.stack([per[k][2] for k in keys], 1)
    md = np.where((LO >= 0) & (LO == UP), LO, -1)
    crossed = np.isfinite(S) & (LO >= 0)
    order = np.argsort(S, axis=1)
    edges = set()
    off, tgt = geom.map_offsets, geom.map_targets
    n_pairs = 0
    for t in range(pt.size):
        seq = [md[t, j] for j in order[t] if crossed[t, j]]
        for a, b in zip(seq[:-1], seq[1:]):
            if a >= 0 and b >= 0:
                n_pairs += 1
                row = tgt[off[a]:off[a + 1]]
                assert b in row, f"track {t}: MD modules {a} -> {b} not linked"
    assert n_pairs > 10000


# ------------------------------------------------------------- closed forms
def _closed_form_tracks(geom, eta_max, n, seed):
    pt, eta, phi, z0, q = _tracks(n, seed, eta_max)
    pt[: n // 8] = 0.8 + 1e-4 * np.arange(n // 8)  # at the threshold
    return pt, eta, phi, z0, q


def _chain_counts(geom, mds):
    """Number of chains of k MDs (k = 2, 3, 5) with consecutive members linked by the map."""
    off, tgt = geom.map_offsets, geom.map_targets
    n = len(mds)
    link = [[j for j in range(i + 1, n) if mds[j] in tgt[off[mds[i]]:off[mds[i] + 1]]] for i in range(n)]
    ways = [[1] * n]
    for _ in range(4):
        prev = ways[-1]
        ways.append([sum(prev[j] for j in link[i]) for i in range(n)])
    return {2: sum(ways[1]), 3: sum(ways[2]), 5: sum(ways[4])}


@pytest.mark.parametrize("which,eta_max", [("barrel", 0.5), ("full", 2.4)])
def test_single_track_closed_form(which, eta_max, barrel, full, obarrel, ofull):
    """Closed form: a noise-free single-track event yields exactly one quintuplet per track."""
    geom, og = (barrel, obarrel) if which == "barrel" else (full, ofull)
    pt, eta, phi, z0, q = _closed_form_tracks(geom, eta_max, 48, 31 if which == "barrel" else 32)
    n_eligible = 0
    for i in range(pt.size):
        cr = md_surfaces(geom, pt[i], eta[i], phi[i], z0[i], 0.0, q[i])
        ev = make_single_track_event(geom, pt[i], eta[i], phi[i], z0=z0[i], d0=0.0, q=q[i])
        r = oracle.run(og, ev, last=oracle.ST_T5)
        mds = [c[2] for c in cr if c[2] >= 0]
        assert r.count(oracle.ST_MD) == len(mds)
        # chains of map-linked MDs of this track, in crossing order (exact hits pass every cut)
        chains = _chain_counts(geom, mds)
        assert r.count(oracle.ST_LS) == chains[2]
        assert r.count(oracle.ST_T3) == chains[3]
        assert r.count(oracle.ST_T5) == chains[5]
        _, keep, _ = r.stage(oracle.ST_T5)
        # any two 5-MD chains out of at most 8 MDs share two MDs: one T5 survives
        assert len(mds) <= 8
        assert keep.sum() == (1 if chains[5] else 0)
        n_eligible += chains[5] > 0
    assert n_eligible >= pt.size // 2


def test_attributes_closed_form(full, ofull):
    """kappa3 = kappa5 = -qK/pT; chi2 = 0; beta_in/out = asin(kappa r/2) at the other anchor."""
    pt, eta, phi, z0, q = _closed_form_tracks(full, 1.2, 24, 41)
    for i in range(pt.size):
        for d0 in (0.0, 0.05):
            ev = make_single_track_event(full, pt[i], eta[i], phi[i], z0=z0[i], d0=d0, q=q[i])
            r = oracle.run(ofull, ev, last=oracle.ST_T5)
            kt = kappa_true(pt[i], q[i])
            _, _, a3 = r.stage(oracle.ST_T3)
            assert np.all(np.abs(a3[:, 0] - kt) < 2e-6)
            assert np.all(a3[:, 2] < 1e-3)
            _, _, a5 = r.stage(oracle.ST_T5)
            assert np.all(np.abs(a5[:, 0] - kt) < 3e-6)
            assert np.all(a5[:, 1] < 1e-3) and np.all(a5[:, 2] < 1e-3)
            assert np.all(np.abs(a5[:, 3] - np.sinh(eta[i])) < 1e-3 * (1 + abs(np.sinh(eta[i]))))
            if d0 == 0.0:
                tl, _, al = r.stage(oracle.ST_LS)
                ra = np.hypot(ev.x[tl[:, 0]], ev.y[tl[:, 0]]).astype(np.float64)
                rb = np.hypot(ev.x[tl[:, 2]], ev.y[tl[:, 2]]).astype(np.float64)
                assert np.all(np.abs(al[:, 0] - np.arcsin(kt * rb / 2)) < 2e-5)
                assert np.all(np.abs(al[:, 1] - np.arcsin(kt * ra / 2)) < 2e-5)


def test_below_threshold_makes_no_md(barrel, obarrel):
    """Section 2.2: the MD window is the pT threshold; a 0.5 GeV track forms no MD."""
    for phi in np.linspace(0.1, 6.0, 12):
        for q in (-1, 1):
            ev = make_single_track_event(barrel, 0.5, 0.2, phi, z0=2.0, q=q)
            assert ev.n_hits >= 8
            r = oracle.run(obarrel, ev, last=oracle.ST_MD)
            assert r.count(oracle.ST_MD) == 0


# ----------------------------------------------------------- library routine
def test_t5_circle_fit_equals_lstsq(barrel, obarrel):
    """The 5-anchor circle fit (Cramer's rule, FP32) equals numpy's weighted lstsq (FP64)."""
    og64 = oracle.OracleGeometry(barrel, f64=True)
    n_checked = 0
    for seed in range(3):
        ev = make_event("tiny", seed)
        for og, tol in ((obarrel, 2e-3), (og64, 1e-9)):
            r = oracle.run(og, ev, last=oracle.ST_T5)
            tup, _, attr = r.stage(oracle.ST_T5)
            for k in range(min(len(tup), 60)):
                lo = tup[k, 0::2]
                X = ev.x[lo].astype(np.float64)
                Y = ev.y[lo].astype(np.float64)
                ty = barrel.type[ev.module[lo]]
                sig = np.where(ty == 0, 0.005, 0.0045)
                ex, ey = X[4] - X[0], Y[4] - Y[0]
                L = math.hypot(ex, ey)
                ux, uy = ex / L, ey / L
                u = ((X - X[0]) * ux + (Y - Y[0]) * uy) / L
                v = ((Y - Y[0]) * ux - (X - X[0]) * uy) / L
                qq = u * u + v * v
                sw = L / sig
                A = np.stack([np.ones(5), u, qq], 1) * sw[:, None]
                coef, *_ = np.linalg.lstsq(A, v * sw, rcond=None)
                res = v - A.dot(coef) / sw
                chi2 = float(np.sum((res * sw) ** 2))
                a, b, c = coef
                k5 = 2 * c / (L * math.sqrt(1 + b * b - 4 * a * c))
                assert abs(attr[k, 0] - k5) <= tol * abs(k5) + (1e-7 if og is obarrel else 1e-13)
                assert abs(attr[k, 1] - chi2) <= tol * chi2 + (2e-3 if og is obarrel else 1e-9)
                n_checked += 1
    assert n_checked > 100


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(6))
def test_staged_equals_brute_force(seed, obarrel):
    ev = make_tiny_event(seed, n_tracks=10, n_noise=20)
    r = oracle.run(obarrel, ev, last=oracle.ST_T5)
    b, counts = oracle.run_brute(obarrel, ev)
    for st in (oracle.ST_MD, oracle.ST_LS, oracle.ST_T3, oracle.ST_T5):
        ts, fs, as_ = r.stage(st)
        tb, fb, ab = b.stage(st)
        assert np.array_equal(ts, tb), oracle.STAGE_NAMES[st]
        assert np.array_equal(fs, fb)
        assert np.array_equal(as_, ab)
    assert counts[0] > 0 and counts[3] > 0


# ------------------------------------------------------------------ invariance
def _tc_sets(r):
    ty, off, hits = r.tc()
    return sorted((int(t), tuple(hits[off[i]:off[i + 1]])) for i, t in enumerate(ty))


def test_hit_relabelling_invariance(obarrel):
    ev = make_event("tiny", 3)
    r1 = oracle.run(obarrel, ev)
    perm = np.random.Generator(np.random.PCG64(9)).permutation(ev.n_hits)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    ev2 = Event(x=ev.x[perm], y=ev.y[perm], z=ev.z[perm], module=ev.module[perm], sensor=ev.sensor[perm],
                sim=ev.sim[perm])
    r2 = oracle.run(obarrel, ev2)
    a = sorted((t, tuple(sorted(h))) for t, h in _tc_sets(r1))
    b = sorted((t, tuple(sorted(perm[list(h)]))) for t, h in _tc_sets(r2))
    assert a == b
    assert len(a) > 50


# ------------------------------------------------------------ cleaning fixtures
def _seeded(geom, pts, etas, phis, qs, z0=0.0):
    return make_single_track_event(geom, pts, etas, phis, z0=z0, q=qs, seeded=True)


def test_tc_single_seeded_track_is_one_pt5(barrel, obarrel):
    ev = _seeded(barrel, 3.0, 0.1, 0.7, 1)
    assert ev.n_seeds == 1
    r = oracle.run(obarrel, ev)
    ty, off, hits = r.tc()
    assert list(ty) == [0]
    assert off[1] == 14
    assert list(hits[:4]) == list(ev.hits4[0])
    t5, k5, _ = r.stage(oracle.ST_T5)
    assert list(hits[4:]) == list(t5[k5 == 1][0])


def test_tc_duplicate_seed(barrel, obarrel):
    """Same pixel hits twice: pLS duplicate removal and pT5 duplicate removal keep seed 0 only."""
    ev = _seeded(barrel, 3.0, 0.1, 0.7, 1)
    for f in ("px", "py", "pz", "q", "seed_sim"):
        setattr(ev, f, np.concatenate([getattr(ev, f), getattr(ev, f)]))
    ev.hits4 = np.concatenate([ev.hits4, ev.hits4])
    r = oracle.run(obarrel, ev)
    ty, off, hits = r.tc()
    assert list(ty) == [0]
    t5, f5, _ = r.stage(oracle.ST_PT5)
    assert list(t5[f5 == 1][:, 0]) == [0]
    _, fp, _ = r.stage(oracle.ST_PLS)
    assert list(fp) == [1, 0]


def _drop_layers(ev, geom, layers):
    keep = np.ones(ev.n_hits, bool)
    outer = ev.module >= 0
    keep[outer] = ~np.isin(geom.layer[ev.module[outer]], layers) | (geom.subdet[ev.module[outer]] != 0)
    new_index = np.cumsum(keep) - 1
    ev2 = Event(x=ev.x[keep], y=ev.y[keep], z=ev.z[keep], module=ev.module[keep], sensor=ev.sensor[keep],
                sim=ev.sim[keep], px=ev.px, py=ev.py, pz=ev.pz, q=ev.q,
                hits4=new_index[ev.hits4].astype(np.int32), seed_sim=ev.seed_sim)
    return ev2


def test_tc_four_layers_is_pt3(barrel, obarrel):
    ev = _drop_layers(_seeded(barrel, 3.0, 0.1, 0.7, 1), barrel, [5, 6])
    r = oracle.run(obarrel, ev)
    ty, off, _ = r.tc()
    assert list(ty) == [1] and off[1] == 10


def test_tc_unseeded_track_is_t5(barrel, obarrel):
    ev = make_single_track_event(barrel, 3.0, 0.1, 0.7, q=1)
    r = oracle.run(obarrel, ev)
    ty, off, _ = r.tc()
    assert list(ty) == [2] and off[1] == 10


def test_tc_bare_seed_is_pls(barrel, obarrel):
    ev = _drop_layers(_seeded(barrel, 3.0, 0.1, 0.7, 1), barrel, [1, 2, 3, 4, 5, 6])
    r = oracle.run(obarrel, ev)
    ty, off, _ = r.tc()
    assert list(ty) == [3] and off[1] == 4


@pytest.mark.parametrize("dphi,expect", [(0.004, [0]), (0.2, [0, 1])])
def test_tc_pt3_near_pt5_is_cleaned(dphi, expect, barrel, obarrel):
    """Section 2.5: a pT3 near (eta-phi) a pT5 is not added; a far one is."""
    full_ev = _seeded(barrel, 3.0, 0.1, 0.7, 1)
    short = _drop_layers(_seeded(barrel, 3.0, 0.1, 0.7 + dphi, 1), barrel, [5, 6])
    n1 = full_ev.n_hits
    ev = Event(x=np.concatenate([full_ev.x, short.x]), y=np.concatenate([full_ev.y, short.y]),
               z=np.concatenate([full_ev.z, short.z]), module=np.concatenate([full_ev.module, short.module]),
               sensor=np.concatenate([full_ev.sensor, short.sensor]), sim=np.concatenate([full_ev.sim, short.sim]),
               px=np.concatenate([full_ev.px, short.px]), py=np.concatenate([full_ev.py, short.py]),
               pz=np.concatenate([full_ev.pz, short.pz]), q=np.concatenate([full_ev.q, short.q]),
               hits4=np.concatenate([full_ev.hits4, short.hits4 + n1]).astype(np.int32),
               seed_sim=np.array([0, 1], np.int32))
    r = oracle.run(obarrel, ev)
    ty, _, _ = r.tc()
    assert sorted(ty) == expect


# ---------------------------------------------------------------- FP64 shadow
def test_fp64_shadow_agrees_on_tiny(barrel, obarrel):
    og64 = oracle.OracleGeometry(barrel, f64=True)
    for seed in range(3):
        ev = make_event("tiny", seed)
        a = oracle.run(obarrel, ev)
        b = oracle.run(og64, ev)
        for st in range(oracle.ST_TC):
            ta = {tuple(t) for t in a.stage(st)[0]}
            tb = {tuple(t) for t in b.stage(st)[0]}
            assert len(ta ^ tb) <= max(1, len(ta) // 1000), oracle.STAGE_NAMES[st]
