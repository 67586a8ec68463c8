"""A dense seeded fixture: single tracks whose outer hits are repeated a few times within the
pitch, so that every module holds k x k mini-doublets of one trajectory and the seed of the track
finds hundreds to thousands of compatible triplets and tens of surviving quintuplets (the
seed-search cases above the per-seed caches and the LDS list)."""
import numpy as np

from lstgen import make_single_track_event
from lstgen.events import Event
from lstgen.geometry import PITCH

# (pT, eta, phi, charge, copies per sensor hit, barrel layers kept)
TRACKS = [
    (2.0, 0.1, 0.7, 1, 3, (1, 2, 3, 4)),       # ~1,458 triplets on one trajectory
    (2.0, -0.2, 2.5, -1, 3, (1, 2, 3)),        # ~729
    (2.0, 0.3, 4.5, 1, 2, (1, 2, 3, 4, 5)),    # 1,024 quintuplets, many of them disjoint
]


def _copies(x, y, z, ptype, k):
    """k copies of one hit, spread along the sensor within 40% of a half pitch."""
    r = np.hypot(x, y)
    out = []
    for j in range(k):
        f = (j - (k - 1) / 2.0) / max(1, k - 1) * 0.4
        a = f * PITCH[ptype][0] / 2 / r
        c, s = np.cos(a), np.sin(a)
        out.append((c * x - s * y, s * x + c * y, z + f * min(PITCH[ptype][1], 0.15) / 2))
    return out


def dense_event(geom, tracks=TRACKS):
    xs, ys, zs, mods, sens, sims = [], [], [], [], [], []
    px, py, pz, q, h4 = [], [], [], [], []
    for ti, (pt, eta, phi, ch, k, layers) in enumerate(tracks):
        ev = make_single_track_event(geom, pt, eta, phi, z0=0.0, q=ch, seeded=True)
        base = len(xs)
        for h in range(4):  # pixel hits of the seed
            i = ev.hits4[0][h]
            xs.append(ev.x[i]); ys.append(ev.y[i]); zs.append(ev.z[i])
            mods.append(-1); sens.append(0); sims.append(ti)
        h4.append([base, base + 1, base + 2, base + 3])
        px.append(ev.px[0]); py.append(ev.py[0]); pz.append(ev.pz[0]); q.append(ev.q[0])
        for i in range(ev.n_hits):
            m = int(ev.module[i])
            if m < 0 or geom.subdet[m] != 0 or geom.layer[m] not in layers:
                continue
            for (x, y, z) in _copies(float(ev.x[i]), float(ev.y[i]), float(ev.z[i]), int(geom.type[m]), k):
                xs.append(x); ys.append(y); zs.append(z)
                mods.append(m); sens.append(int(ev.sensor[i])); sims.append(ti)
    f = lambda v: np.asarray(v, np.float32)
    i = lambda v: np.asarray(v, np.int32)
    return Event(x=f(xs), y=f(ys), z=f(zs), module=i(mods), sensor=i(sens), sim=i(sims), px=f(px), py=f(py),
                 pz=f(pz), q=i(q), hits4=i(h4), seed_sim=np.arange(len(tracks), dtype=np.int32), name="dense")


def spread_event(geom):
    """Nine tracks 3 mrad apart (pT 1 GeV, two copies of every hit, barrel layers 1-5), seeded only
    in the middle: that seed makes pT5 with 18 surviving quintuplets and pT3 with ~21,000
    triplets."""
    tr = [(1.0, 0.3, 4.5 + 0.003 * j, 1, 2, (1, 2, 3, 4, 5)) for j in range(-4, 5)]
    ev = dense_event(geom, tr)
    k = [4]
    ev.px, ev.py, ev.pz, ev.q = ev.px[k], ev.py[k], ev.pz[k], ev.q[k]
    ev.hits4, ev.seed_sim = ev.hits4[k], np.zeros(1, np.int32)
    ev.name = "dense-spread"
    return ev
