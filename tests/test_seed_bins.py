"""The seed search visits only the first-anchor bins its seed marks (Section 2.4's
window at the first anchor): every (ring, azimuth) bin within reach of the seed
trajectory, sampled every 2 cm of arc, and per ring the z bins its slope
allows.  The marking must hold the first anchor of every pT3 and pT5 the exact
selection accepts.  This replays the kernels' marking in float32 on the host
(seed parameters as the pLS step forms them, sample positions, the azimuth
run asin(d / (r - d)) either side with its 2e-4 rad rounding margin, the rings
within d, the z bins from the arc-length range of the ring's samples) and
checks on a PU200-like event that the first anchor of every pT3 and pT5 of the
oracle, which searches all objects without bins, lies in a marked bin of its
seed.  A missing margin term or a wrong sign leaves anchors outside.
"""
import numpy as np
import pytest

import oracle
from lstgen.events import make_event, geometry_for

f32 = np.float32
K_CURV = f32(0.299792458 * 3.8 / 100.0)
K_BOX_XY, K_BOX_Z0 = f32(1.0), f32(3.0)
K_RINGS, K_RING0, K_RING_W = 10, f32(20.0), f32(10.0)
K_PHI_BINS = 256
K_ZBINS, K_ZHALF, K_ZW = 55, f32(275.0), f32(10.0)
K_STEP, K_MAX_SAMPLES = f32(2.0), 112
PI = f32(np.pi)


def ring_of(r):
    return np.clip(np.floor((r - K_RING0) / K_RING_W).astype(np.int64), 0, K_RINGS - 1)


def phibin_of(ph):
    return np.clip(np.floor((ph + PI) * f32(K_PHI_BINS / (2.0 * np.pi))).astype(np.int64), 0, K_PHI_BINS - 1)


def zbin_of(z):
    return np.clip(np.floor((z + K_ZHALF) / K_ZW).astype(np.int64), 0, K_ZBINS - 1)


def seeds_of(ev):
    """Seed parameters as the pLS step forms them: pT, direction, slope, curvature, first pixel hit."""
    px, py, pz = ev.px.astype(f32), ev.py.astype(f32), ev.pz.astype(f32)
    pt = np.sqrt(px * px + py * py)
    h0 = np.asarray(ev.hits4, np.int64).reshape(-1, 4)[:, 0]
    return dict(cx=px / pt, cy=py / pt, lam=pz / pt, ks=(-ev.q.astype(f32) * K_CURV) / pt,
                x0=ev.x.astype(f32)[h0], y0=ev.y.astype(f32)[h0], z0=ev.z.astype(f32)[h0])


def marked(sd, s):
    """(mask [rings, phi bins] bool, z-bin range per ring [rings, 2]) of seed s."""
    cx, cy, lam, k = sd["cx"][s], sd["cy"][s], sd["lam"][s], sd["ks"][s]
    x0, y0, z0 = sd["x0"][s], sd["y0"][s], sd["z0"][s]
    d = f32(1.01) * K_BOX_XY + f32(0.5) * K_STEP + f32(0.05)
    bw = f32(2.0 * np.pi / K_PHI_BINS)
    ak = max(abs(k), f32(1e-9))
    s_max = PI / ak
    sarc = np.arange(K_MAX_SAMPLES, dtype=f32) * K_STEP
    sarc = sarc[~(sarc > s_max + K_STEP)]
    a = k * sarc
    if abs(k) > 1e-9:
        s1 = np.sin(a) / k
        sh = np.sin(f32(0.5) * a)
        s2 = f32(2.0) * sh * sh / k
    else:
        s1, s2 = sarc, np.zeros_like(sarc)
    x = x0 + cx * s1 + (-cy) * s2
    y = y0 + cy * s1 + cx * s2
    r = np.sqrt(x * x + y * y)
    keep = ~((r + d < K_RING0 - 5) | (r - d > K_RING0 + K_RINGS * K_RING_W + 5))
    mask = np.zeros((K_RINGS, K_PHI_BINS), bool)
    lo = np.full(K_RINGS, np.inf, f32)
    hi = np.full(K_RINGS, -np.inf, f32)
    for xi, yi, ri, si in zip(x[keep], y[keep], r[keep], sarc[keep]):
        r0, r1 = int(ring_of(ri - d)), int(ring_of(ri + d))
        rin = ri - d
        if rin <= 1e-3 or d / rin >= 1.0:
            b0, b1 = 0, K_PHI_BINS - 1
        else:
            hw = np.arcsin(d / rin)
            ph = np.arctan2(yi, xi)
            b0 = int(np.floor((ph - hw - f32(2e-4) + PI) / bw))
            b1 = int(np.floor((ph + hw + f32(2e-4) + PI) / bw))
            if b1 - b0 >= K_PHI_BINS:
                b0, b1 = 0, K_PHI_BINS - 1
        bins = np.arange(b0, b1 + 1) % K_PHI_BINS
        for rr in range(r0, r1 + 1):
            mask[rr, bins] = True
            lo[rr] = min(lo[rr], si)
            hi[rr] = max(hi[rr], si)
    ds = f32(1.01) * K_BOX_XY + f32(1.5) * K_STEP + f32(1.6)
    zw = (K_BOX_Z0 + f32(2.0) * max(f32(2.5), f32(2.5) * abs(lam) + f32(0.01))) * f32(1.01) + f32(0.1)
    za, zb = z0 + lam * (lo - ds), z0 + lam * (hi + ds)
    with np.errstate(invalid="ignore"):
        zr = np.stack([zbin_of(np.minimum(za, zb) - zw), zbin_of(np.maximum(za, zb) + zw)], 1)
    return mask, zr


@pytest.fixture(scope="module")
def pt_objects():
    geom = geometry_for("pu200_seeded")
    ev = make_event("pu200_seeded", 4)
    r = oracle.run(oracle.OracleGeometry(geom), ev, last=6)
    t3, _, _ = r.stage(5)
    t5, _, _ = r.stage(6)
    return ev, t3, t5


def test_every_pt_first_anchor_is_in_a_marked_bin(pt_objects):
    ev, t3, t5 = pt_objects
    sd = seeds_of(ev)
    x, y, z = ev.x.astype(f32), ev.y.astype(f32), ev.z.astype(f32)
    seeds = np.concatenate([t3[:, 0], t5[:, 0]])
    anchors = np.concatenate([t3[:, 1], t5[:, 1]])  # the lower hit of the first MD
    assert len(t3) > 20000 and len(t5) > 500
    ax, ay, az = x[anchors], y[anchors], z[anchors]
    ring = ring_of(np.sqrt(ax * ax + ay * ay))
    phib = phibin_of(np.arctan2(ay, ax))
    zb = zbin_of(az)
    order = np.argsort(seeds, kind="stable")
    missed = []
    cur, mask, zr = -1, None, None
    for i in order:
        s = int(seeds[i])
        if s != cur:
            mask, zr = marked(sd, s)
            cur = s
        if not (mask[ring[i], phib[i]] and zr[ring[i], 0] <= zb[i] <= zr[ring[i], 1]):
            missed.append((s, int(anchors[i])))
    assert not missed, f"{len(missed)} first anchors outside their seed's bins, e.g. {missed[:3]}"
