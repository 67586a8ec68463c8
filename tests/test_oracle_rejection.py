"""Rejection side of the oracle's selections (Sections 2.2-2.4) and the
cleaning rules of Section 2.5, pinned to constructions that do not come from
the oracle.

Every selection is evaluated on hand-placed hits through the oracle's own
predicate (``oracle.probe_*``), which reports each cut it evaluated as
(quantity, bound).  For each cut the test builds, in float64 from the
generator's exact helices and the stated error model, the configuration at
the edge of what the cut is meant to admit (the pT-threshold helix, the
impact-parameter bound, the luminous-region edge, half-pitch displacements
of the hits, a chi2 equal to its cut) and checks that

* the edge configuration passes the cut,
* the same configuration moved a little beyond the edge fails that cut,
* where the cut has no designed slack, its bound equals the edge within the
  selections' stated safety margin (1e-3 relative + a small absolute term),
  and where it has slack (an upper-bound expression), within that slack;
* the cut's quantity equals an independent closed form (circumcircle
  curvature, numpy least squares, straight-line extrapolation).

A sign error, a dropped or doubled error term, a transposed operand or a
wrong category index moves a boundary outside these bands.
"""
import math

import numpy as np
import pytest

import oracle
from lstgen import make_single_track_event
from lstgen.events import Event
from lstgen.geometry import BARREL_RADII, K_CURV, PT_MIN, cylinder_s, helix_point, plane_s

KM = K_CURV / PT_MIN            # curvature at the pT threshold [1/cm]
D0 = 0.1                        # default impact-parameter bound [cm]
ZL = 20.0                       # luminous-region half length [cm]
HP = {0: 0.005, 1: 0.0045}      # half pitch across the strip (r-phi), PS / 2S [cm]
HL = {0: 0.075, 1: 2.5}         # half pitch along the strip, PS / 2S [cm]
MARGIN = 1e-3                   # relative safety margin every window carries


# ------------------------------------------------------------------ helpers
def at_r(phi0, d0, z0, kap, lam, r):
    """Exact crossing of radius r by the helix (outgoing half-turn)."""
    s = cylinder_s(np.array([d0]), np.array([kap]), r)[0]
    assert np.isfinite(s)
    return np.array(helix_point(phi0, d0, z0, kap, lam, s), np.float64)


def at_z(phi0, d0, z0, kap, lam, zp):
    s = plane_s(np.array([z0]), np.array([kap]), np.array([lam]), zp)[0]
    assert np.isfinite(s)
    return np.array(helix_point(phi0, d0, z0, kap, lam, s), np.float64)


def rot(p, a):
    """Point p rotated by angle a about the beam line."""
    c, s = math.cos(a), math.sin(a)
    return np.array([c * p[0] - s * p[1], s * p[0] + c * p[1], p[2]])


def scale_r(p, r_new):
    """Point p moved radially to transverse radius r_new."""
    f = r_new / math.hypot(p[0], p[1])
    return np.array([p[0] * f, p[1] * f, p[2]])


def dphi(a, b):
    """Signed azimuth from point a to point b."""
    return math.atan2(a[0] * b[1] - a[1] * b[0], a[0] * b[0] + a[1] * b[1])


def f32(p):
    return np.asarray(p, np.float32).astype(np.float64)


def rxy(p):
    p = f32(p)
    return math.hypot(p[0], p[1])


def bmod(g, li, phi, z):
    R = BARREL_RADII[li]
    m = int(g.lookup("b", li, 0, [R * math.cos(phi)], [R * math.sin(phi)], [z])[0])
    assert m >= 0
    return m


def emod(g, disk, side, r, phi):
    m = int(g.lookup("e", disk, side, [r * math.cos(phi)], [r * math.sin(phi)], [0.0])[0])
    assert m >= 0
    return m


def linked(g, a, b):
    return b in g.map_targets[g.map_offsets[a]:g.map_offsets[a + 1]]


def curvature(a, b, c):
    """Signed curvature of the circle through three points (x-y), counter-clockwise positive."""
    ax, ay = b[0] - a[0], b[1] - a[1]
    bx, by = c[0] - a[0], c[1] - a[1]
    cross = ax * by - ay * bx
    la, lb, lc = math.hypot(ax, ay), math.hypot(bx, by), math.hypot(c[0] - b[0], c[1] - b[1])
    return 2.0 * cross / (la * lb * lc)


def bisect(f, lo, hi, n=60):
    """Point where the predicate f flips from True (at lo) to False (at hi)."""
    assert f(lo) and not f(hi)
    for _ in range(n):
        mid = 0.5 * (lo + hi)
        if f(mid):
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.fixture(scope="module")
def og(full):
    return oracle.OracleGeometry(full)


@pytest.fixture(scope="module")
def og_wide(full):
    """The same detector with a 5 cm impact-parameter bound: the azimuth-z test then admits any z
    displacement used below, so the chi2 cuts behind it can be reached."""
    return oracle.OracleGeometry(full, d0_max=5.0)


# ----------------------------------------------------------------------- MD
def _md_barrel_edge(g, li, phi=0.3, z=2.5):
    """Largest azimuth change between the two sensors of a barrel module admitted by the
    hypothesis: a threshold helix (either charge) with |d0| at its bound, each hit rotated by
    its half pitch.  Returns (module, r_lo, r_up, signed helix change, full edge angle)."""
    m = bmod(g, li, phi, z)
    r1, r2 = g.pos_lo[m], g.pos_up[m]
    best = 0.0
    for q in (-1, 1):
        for d0 in (-D0, D0):
            a = at_r(phi, d0, 0.0, -q * KM, 0.0, r1)
            b = at_r(phi, d0, 0.0, -q * KM, 0.0, r2)
            d = dphi(a, b)
            if abs(d) > abs(best):
                best = d
    hp = HP[int(g.type[m])]
    return m, r1, r2, best, abs(best) + hp / r1 + hp / r2


@pytest.mark.parametrize("li", [0, 3])
def test_md_azimuth_window_is_the_threshold_edge(li, full, og):
    """MD x-y (Section 2.2): the window is exactly the threshold helix at the d0 bound plus one
    half pitch per hit (PS and 2S barrel modules)."""
    m, r1, r2, hel, D = _md_barrel_edge(full, li)
    sg = math.copysign(1.0, hel)
    lo = np.array([r1 * math.cos(0.3), r1 * math.sin(0.3), 2.5])
    for f, ok in ((1.0, True), (1.0 + 2.5 * MARGIN, False)):
        up = rot(np.array([r2 * math.cos(0.3), r2 * math.sin(0.3), 2.5]), sg * D * f)
        p = oracle.probe_md(og, m, lo, up)
        assert p.ok == ok and p.passes(0) == ok and p.failing() == ([] if ok else [0])
        # quantity: r_lo r_up |sin(azimuth change)| of the float hits
        qf = rxy(lo) * rxy(up) * abs(math.sin(dphi(f32(lo), f32(up))))
        assert abs(p.cuts[0][0] - qf) <= 2e-4 * qf
    # the boundary: sin(edge) = bound / (r_lo r_up), within the window's stated margin
    q, b, _ = p.cuts[0]
    flip = math.asin(b / (rxy(lo) * rxy(up)))
    assert D * (1 - 1e-5) <= flip <= D * (1 + MARGIN) + 1.1e-6 + 1e-5 * D
    # each term of the window is larger than that band: dropping or doubling it moves the flip out
    band = MARGIN + 1e-5 + 1.1e-6 / D
    hp = HP[int(full.type[m])]
    terms = [hp / r1 + hp / r2, abs(hel) - D0 * (1 / r1 - 1 / r2)]
    if li == 0:  # the impact-parameter term shrinks as 1/r^2: visible on the innermost layer
        terms.append(D0 * (1 / r1 - 1 / r2))
    for term in terms:
        assert term / D > 2 * band


def test_md_z_window_barrel_ps(full, og):
    """MD z (PS barrel, Section 2.2): the upper hit's z is that of a straight line from the
    luminous-region edge, stretched by the threshold helix's arc length, plus a half pitch per hit."""
    m = bmod(full, 0, 0.3, 52.0)
    r1, r2 = full.pos_lo[m], full.pos_up[m]
    hl = HL[0]
    s_of = lambda r: 2.0 * math.asin(KM * r / 2.0) / KM
    ap = s_of(r2) / s_of(r1)
    a = r2 / r1
    z_lo = 52.0
    # positive edge: z0 = -20, threshold curvature, the pitch pushing both hits apart
    z_lo_true = z_lo + hl
    z_up = (-ZL + (z_lo_true + ZL) * ap) + hl
    t_edge = z_up - a * z_lo
    lo = np.array([r1 * math.cos(0.3), r1 * math.sin(0.3), z_lo])
    up = lambda zz: np.array([r2 * math.cos(0.3), r2 * math.sin(0.3), zz])
    p = oracle.probe_md(og, m, lo, up(z_up))
    assert p.ok and len(p.cuts) == 2
    q, b, _ = p.cuts[1]
    assert abs(q - t_edge) <= 2e-5 * abs(z_up)
    assert t_edge <= b <= t_edge * (1 + MARGIN) + 1e-4
    assert not oracle.probe_md(og, m, lo, up(z_up + 2.5 * MARGIN * b)).passes(1)
    # negative edge: z0 = +20, straight track, pitch pushing the hits together
    z_up_n = (ZL + (z_lo - hl - ZL) * a) - hl
    assert oracle.probe_md(og, m, lo, up(z_up_n)).ok
    # a hit pair that only an impact point outside the luminous region explains fails
    z_far = (-1.05 * ZL + (z_lo_true + 1.05 * ZL) * ap) + hl
    assert not oracle.probe_md(og, m, lo, up(z_far)).passes(1)


def test_md_2s_modules_have_no_long_cut(full, og):
    m = bmod(full, 4, 0.3, 52.0)
    assert full.type[m] == 1
    r1, r2 = full.pos_lo[m], full.pos_up[m]
    p = oracle.probe_md(og, m, [r1 * math.cos(0.3), r1 * math.sin(0.3), 52.0],
                        [r2 * math.cos(0.3), r2 * math.sin(0.3), 54.4])
    assert p.ok and len(p.cuts) == 1


def test_md_endcap_ps_windows(full, og):
    """MD in an endcap PS module (Section 2.2): azimuth and radius windows of a threshold helix
    from the luminous-region edge nearest the disk (the shallowest track), within pitch."""
    side, disk, phi = 1, 0, 0.4
    rmid = 27.0
    m = emod(full, disk, side, rmid, phi)
    assert full.type[m] == 0 and full.subdet[m] == 1
    z1, z2 = full.pos_lo[m], full.pos_up[m]
    rmin, rmax = full.lmin[m], full.lmax[m]
    hl, hp = HL[0], HP[0]
    # the shallowest threshold track reaching r = rmax at the lower plane starts at z0 = +20
    s1 = 2.0 * math.asin(KM * rmax / 2.0) / KM
    lam = (z1 - ZL) / s1
    best = None
    for q in (-1, 1):
        a = at_z(0.0, 0.0, ZL, -q * KM, lam, z1)
        b = at_z(0.0, 0.0, ZL, -q * KM, lam, z2)
        best = (a, b)
    a, b = best
    dr_true = math.hypot(b[0], b[1]) - math.hypot(a[0], a[1])
    hel = abs(dphi(a, b))
    # radius window, upper edge: lower hit pulled in by hl, upper pushed out
    lo = scale_r(a, math.hypot(a[0], a[1]) - hl)
    lo = rot(lo, 0.0)
    up = scale_r(b, math.hypot(b[0], b[1]) + hl)
    p = oracle.probe_md(og, m, lo, up)
    assert p.ok and len(p.cuts) == 3
    dr_edge = dr_true + 2 * hl
    q, bnd, _ = p.cuts[2]
    assert abs(q - dr_edge) <= 1e-5
    # the window's growth factor bounds the radius change by arc length (>= the radial change),
    # a slack of 1 / cos(crossing angle) on the helix part, ~2% on the innermost ring
    slack = 1.0 / math.sqrt(1.0 - (KM * rmax / 2.0) ** 2)
    assert dr_edge <= bnd <= (dr_true * slack + 2 * hl + dr_true * hl / rmin) * (1 + MARGIN) + 1e-5
    up_far = scale_r(b, math.hypot(b[0], b[1]) + hl + 1.5 * (bnd - dr_edge) + 1e-3)
    assert not oracle.probe_md(og, m, lo, up_far).passes(2)
    # radius window, lower edge: no radial change, pitch pulling the hits together
    lo2 = scale_r(a, math.hypot(a[0], a[1]) + hl)
    up2 = scale_r(a, math.hypot(a[0], a[1]) - hl)
    up2[2] = z2
    p2 = oracle.probe_md(og, m, lo2, up2)
    assert p2.passes(1)
    q2, b2, _ = p2.cuts[1]
    assert abs(q2 - 2 * hl) <= 1e-5 and 2 * hl <= b2 <= 2 * hl * (1 + 0.01)
    up3 = scale_r(a, math.hypot(a[0], a[1]) - hl - 0.02 * hl)
    up3[2] = z2
    assert not oracle.probe_md(og, m, lo2, up3).passes(1)
    # azimuth window: helix change at rmax + impact-parameter and pitch terms at rmin
    dw = lambda ang: oracle.probe_md(og, m, lo, rot(up, ang))
    W_flip = bisect(lambda ang: dw(ang).passes(0), 0.0, 0.05)
    edge = hel + 2 * hp / rmin
    assert edge <= W_flip + dphi(f32(lo), f32(up)) + 1e-6
    assert W_flip + dphi(f32(lo), f32(up)) <= (edge * slack + D0 * (dr_true / rmax) * 2 / rmin) * (1 + MARGIN) + 2e-6


# ----------------------------------------------------------------------- LS
def _ls_hits(g, phi0, d0, z0, kap, lam, surf_a, surf_b):
    """Lower and upper hits of two MDs of one helix on two surfaces ((kind, index, side)),
    with their modules."""
    out, mods = [], []
    for kind, idx, side in (surf_a, surf_b):
        pts = []
        for sensor in (0, 1):
            if kind == "b":
                pos = BARREL_RADII[idx] + (0.13 if sensor else -0.13)
                pts.append(at_r(phi0, d0, z0, kap, lam, pos))
            else:
                from lstgen.geometry import DISK_Z
                pos = side * (DISK_Z[idx] + (0.13 if sensor else -0.13))
                pts.append(at_z(phi0, d0, z0, kap, lam, pos))
        m = int(g.lookup(kind, idx, side, [pts[0][0]], [pts[0][1]], [pts[0][2]])[0])
        assert m >= 0
        out += pts
        mods.append(m)
    assert linked(g, mods[0], mods[1])
    return out, mods


def _rot_md(h, k, ang):
    """Rotates both hits of MD k by ang (a tangential displacement of the module's hits)."""
    h = list(h)
    h[2 * k], h[2 * k + 1] = rot(h[2 * k], ang), rot(h[2 * k + 1], ang)
    return h


@pytest.mark.parametrize("where", ["barrel", "endcap"])
def test_ls_azimuth_window(where, full, og, og_wide):
    """LS x-y (Section 2.2): the azimuth change between the two anchors is bounded by the
    threshold helix at the d0 bound plus a half pitch per anchor; the window's upper-bound form of
    the arc sine (mean-value bound) is its only slack."""
    if where == "barrel":
        sa, sb, lam, phi = ("b", 0, 0), ("b", 1, 0), 0.1, 0.3
    else:
        sa, sb, lam, phi = ("e", 0, 1), ("e", 1, 1), math.sinh(2.0), 0.3
    best = None
    for q in (-1, 1):
        for d0 in (-D0, D0):
            h, mods = _ls_hits(full, phi, d0, 0.0, -q * KM, lam, sa, sb)
            d = dphi(h[0], h[2])
            if best is None or abs(d) > abs(best[0]):
                best = (d, h, mods)
    d, h, mods = best
    sg = math.copysign(1.0, d)
    ma, mb = mods
    ty = lambda m: int(full.type[m])
    # endcap anchors: the radius is the long coordinate; the edge has the measured radii drawn
    # together by one half pitch each (the helix ran between the outer true radii)
    if where == "endcap":
        ea, eb = HL[ty(ma)], HL[ty(mb)]
        for k, e in ((0, ea), (1, -eb)):
            for j in (2 * k, 2 * k + 1):
                h[j] = scale_r(h[j], math.hypot(h[j][0], h[j][1]) + e)
    ra, rb = math.hypot(h[0][0], h[0][1]), math.hypot(h[2][0], h[2][1])
    h = _rot_md(_rot_md(h, 0, -sg * HP[ty(ma)] / ra), 1, sg * HP[ty(mb)] / rb)
    D = abs(dphi(h[0], h[2]))
    p = oracle.probe_ls(og, mods, h)
    assert p.ok, p.cuts
    qf = rxy(h[0]) * rxy(h[2]) * abs(math.sin(dphi(f32(h[0]), f32(h[2]))))
    assert abs(p.cuts[1][0] - qf) <= 2e-4 * qf
    flip = bisect(lambda a: oracle.probe_ls(og, mods, _rot_md(h, 1, sg * a)).passes(1), 0.0, 0.2)
    total = D + flip
    # slack of the arc-sine bound: asin'(ub) / asin'(ua) at the true radii
    ua = KM * (ra - (HL[ty(ma)] if where == "endcap" else 0.0)) / 2.0
    ub = KM * (rb + (HL[ty(mb)] if where == "endcap" else 0.0)) / 2.0
    slack = math.sqrt(1 - ua * ua) / math.sqrt(1 - ub * ub)
    assert D * (1 - 1e-5) <= total <= D * slack * (1 + MARGIN) + 2e-6
    # the impact-parameter term, exactly: widening the bound from 0.1 to 5 cm widens the window
    # (a bound on the sine of the azimuth change) by the beam line's offset 4.9 (1/ra - 1/rb)
    flip_w = bisect(lambda a: oracle.probe_ls(og_wide, mods, _rot_md(h, 1, sg * a)).passes(1), 0.0, 0.5)
    widen = math.sin(D + flip_w) - math.sin(total)
    expect = (5.0 - D0) * (1 / rxy(h[0]) - 1 / rxy(h[2])) * (1 + MARGIN)
    assert abs(widen - expect) <= 2e-3 * expect


def _straight_ls(full, z0, lam, phi=0.3):
    h, mods = _ls_hits(full, phi, 0.0, z0, -1e-7, lam, ("b", 0, 0), ("b", 1, 0))
    return h, mods


@pytest.mark.parametrize("sign", [1, -1])
def test_ls_rz_pointing(sign, full, og):
    """LS r-z (Section 2.2): the straight line through the two anchors, with each anchor's z moved
    by its half pitch, must reach the beam line inside the luminous region; the edge is a straight
    track from z0 = +-20 with the pitch displacements pushing the extrapolation outward."""
    h, mods = _straight_ls(full, sign * ZL, sign * 0.5)
    hl_a, hl_b = HL[int(full.type[mods[0]])], HL[int(full.type[mods[1]])]
    for j in (0, 1):
        h[j] = h[j] + np.array([0, 0, sign * hl_a])
    for j in (2, 3):
        h[j] = h[j] - np.array([0, 0, sign * hl_b])
    ra, rb = rxy(h[0]), rxy(h[2])
    za, zb = f32(h[0])[2], f32(h[2])[2]
    z0_line = (za * rb - zb * ra) / (rb - ra)       # straight-line extrapolation to r = 0
    t = ra / rb
    Ez = (hl_a + t * hl_b) / (1 - t)                # the pitch displacements carried to r = 0
    assert abs(z0_line - sign * (ZL + Ez)) < 2e-3
    p = oracle.probe_ls(og, mods, h)
    assert p.ok, p.cuts
    k = 2 if sign > 0 else 3                         # z0_min <= L and -z0_max <= L
    q, b, _ = p.cuts[k]
    assert abs(q - sign * z0_line) < 2e-3
    assert abs(b - (ZL + Ez) * (1 + MARGIN)) < 1e-4
    shift = (b * (1 + 2 * MARGIN) - q) * (rb - ra) / rb   # moves the extrapolation just past the bound
    h2 = [hh + np.array([0, 0, sign * shift]) if j < 2 else hh for j, hh in enumerate(h)]
    p2 = oracle.probe_ls(og, mods, h2)
    assert not p2.passes(k) and p2.failing() == [k]
    # threshold helices of either charge from the same edge pass (the arc-length range covers them)
    for q_ in (-1, 1):
        hc, mc = _ls_hits(full, 0.3, 0.0, sign * ZL, -q_ * KM, sign * 0.5, ("b", 0, 0), ("b", 1, 0))
        assert oracle.probe_ls(og, mc, hc).ok


def test_ls_stub_directions(full, og):
    """LS stub check (Sections 1, 2.2): each MD's tangential displacement between its two sensors
    equals the one the circle through the beam line and both anchors predicts (exact for a helix
    from the beam line); the check admits the pitch and impact-parameter displacements and fails
    a little beyond them."""
    lam = 0.2
    # quantity, for exact helices through the beam line: the upper hit's tangential offset
    # r_up sin(asin(k r_up / 2) - asin(k r_lo / 2)) less the straight continuation of the track's
    # direction at the lower hit over the sensor gap, (r_up - r_lo) tan(asin(k r_lo / 2))
    for pt in (0.9, 3.0, 40.0):
        for q in (-1, 1):
            kap = -q * K_CURV / pt
            h, mods = _ls_hits(full, 0.3, 0.0, 0.0, kap, lam, ("b", 0, 0), ("b", 1, 0))
            p = oracle.probe_ls(og, mods, h)
            assert p.ok
            for k, md in ((4, 0), (5, 1)):
                r1, r2 = math.hypot(*h[2 * md][:2]), math.hypot(*h[2 * md + 1][:2])
                a1, a2 = math.asin(abs(kap) * r1 / 2), math.asin(abs(kap) * r2 / 2)
                cf = abs(r2 * math.sin(a2 - a1) - (r2 - r1) * math.tan(a1))
                assert abs(p.cuts[k][0] - cf) < 5e-6
    # edge: d0 at its bound and every hit moved by its half pitch, all sign combinations
    worst = []
    h0, mods = _ls_hits(full, 0.3, 0.0, 0.0, -KM, lam, ("b", 0, 0), ("b", 1, 0))
    hp_a, hp_b = HP[int(full.type[mods[0]])], HP[int(full.type[mods[1]])]
    for q in (-1, 1):
        for d0 in (-D0, D0):
            h, _ = _ls_hits(full, 0.3, d0, 0.0, -q * KM, lam, ("b", 0, 0), ("b", 1, 0))
            for signs in np.ndindex(2, 2, 2, 2):
                hh = [rot(h[j], (1 - 2 * signs[j]) * (hp_a if j < 2 else hp_b) / math.hypot(h[j][0], h[j][1]))
                      for j in range(4)]
                p = oracle.probe_ls(og, mods, hh)
                assert p.passes(4) and p.passes(5)
                worst.append((p.cuts[4][0] / p.cuts[4][1], p.cuts[5][0] / p.cuts[5][1], hh))
    # the bound exceeds the largest admitted residual by at most 20% (inner MD; 9% outer), less
    # than any of its terms: two half pitches (the hits), the chord direction's error from the
    # anchors' half pitches and from the impact parameter, carried over the sensor gap
    assert max(w[0] for w in worst) > 0.83 and max(w[1] for w in worst) > 0.92
    # beyond: the upper hit of each MD moved tangentially past the bound fails that MD's check
    for k, md in ((4, 0), (5, 1)):
        hh = max(worst, key=lambda w: w[k - 4])[2]
        j = 2 * md + 1
        r = math.hypot(hh[j][0], hh[j][1])
        p = oracle.probe_ls(og, mods, hh)
        q, b, _ = p.cuts[k]
        flip = bisect(lambda dd: oracle.probe_ls(og, mods, [rot(x, dd / r) if i == j else x
                                                             for i, x in enumerate(hh)]).passes(k), 0.0, 0.2)
        flip_n = bisect(lambda dd: oracle.probe_ls(og, mods, [rot(x, -dd / r) if i == j else x
                                                               for i, x in enumerate(hh)]).passes(k), 0.0, 0.2)
        # one of the two directions adds to the residual: it fails after (bound - residual)
        assert abs(min(flip, flip_n) - (b - q)) < 2e-4 * b + 2e-6


# ---------------------------------------------------------------- T3, phi-z
def _md_hits(g, phi0, d0, z0, kap, lam, layers):
    """Lower and upper hits of one helix on barrel layers (index list), with the modules."""
    h, mods = [], []
    for li in layers:
        lo = at_r(phi0, d0, z0, kap, lam, BARREL_RADII[li] - 0.13)
        up = at_r(phi0, d0, z0, kap, lam, BARREL_RADII[li] + 0.13)
        m = int(g.lookup("b", li, 0, [lo[0]], [lo[1]], [lo[2]])[0])
        assert m >= 0
        h += [lo, up]
        mods.append(m)
    return h, mods


def _sagitta_dir(a, b, c):
    """Unit vector at b, perpendicular to the chord a-c, pointing away from the chord."""
    ex, ey = c[0] - a[0], c[1] - a[1]
    n = np.array([-ey, ex, 0.0]) / math.hypot(ex, ey)
    if np.dot(n, b - a) < 0:
        n = -n
    return n


def test_phiz_residual_and_window(full, og):
    """Azimuth linear in z (Section 2.3, the triplet's further selection): the residual
    sin(dphi_PQ) dz_QR - sin(dphi_QR) dz_PQ of a helix from the beam line is (nearly) zero and is
    linear in a z displacement of the middle anchor.  Its tolerance is the worst case of the hits'
    z and r-phi half pitches (tight: the worst sign combination reaches it), plus the worst case of
    independent beam-line offsets d0 / r at the anchors (exactly linear in the bound)."""
    lam, phi = 0.4, 0.3
    og0 = oracle.OracleGeometry(full, d0_max=1e-9)
    h, mods = _md_hits(full, phi, 0.0, 1.0, -K_CURV / 2.0, lam, [0, 1, 2])
    p = oracle.probe_t3(og, mods, h)
    assert p.ok
    P, Q, R = (f32(h[0]), f32(h[2]), f32(h[4]))
    su, sv = math.sin(dphi(P, Q)), math.sin(dphi(Q, R))
    res0 = su * (R[2] - Q[2]) - sv * (Q[2] - P[2])
    assert abs(p.cuts[1][0] - abs(res0)) < 1e-5
    for dz in (0.05, -0.08, 0.11):
        hh = list(h)
        hh[2] = h[2] + np.array([0, 0, dz])
        hh[3] = h[3] + np.array([0, 0, dz])
        q = oracle.probe_t3(og, mods, hh).cuts[1][0]
        assert abs(q - abs(res0 - (su + sv) * dz)) < 2e-5 * (1 + abs(dz) * 10)
    # impact-parameter part of the tolerance: bound 0.1 cm against (almost) none
    rP, rQ, rR = rxy(P), rxy(Q), rxy(R)
    d0_part = D0 * (abs(R[2] - Q[2]) * abs(1 / rP - 1 / rQ) + abs(Q[2] - P[2]) * abs(1 / rQ - 1 / rR))
    b_d0 = p.cuts[1][1] - oracle.probe_t3(og0, mods, h).cuts[1][1]
    assert abs(b_d0 - d0_part * (1 + MARGIN)) < 1e-4 * d0_part
    # pitch part: the worst sign combination of the z and r-phi half pitches reaches the tolerance
    hl = HL[0]

    def pitched(h, sg):
        hh = list(h)
        for k in range(3):
            a = (1 - 2 * sg[k]) * HP[0] / math.hypot(h[2 * k][0], h[2 * k][1])
            dzk = (1 - 2 * sg[3 + k]) * hl
            hh[2 * k] = rot(h[2 * k], a) + np.array([0, 0, dzk])
            hh[2 * k + 1] = rot(h[2 * k + 1], a) + np.array([0, 0, dzk])
        return hh

    ratios = []
    for sg in np.ndindex(2, 2, 2, 2, 2, 2):
        pr = oracle.probe_t3(og0, mods, pitched(h, sg))
        assert pr.passes(1)
        ratios.append(pr.cuts[1][0] / pr.cuts[1][1])
    assert max(ratios) > 0.95   # the rest: the sine-curvature allowance and the 1e-3 margin
    # the edge with the impact parameter at its bound passes with the default bound
    for q_ in (-1, 1):
        for d0 in (-D0, D0):
            hd, md = _md_hits(full, phi, d0, 1.0, -q_ * K_CURV / 2.0, lam, [0, 1, 2])
            for sg in np.ndindex(2, 2, 2, 2, 2, 2):
                assert oracle.probe_t3(og, md, pitched(hd, sg)).passes(1)
    # beyond: the middle anchor moved in z past the tolerance fails the test, where the linear
    # residual meets the tolerance (which grows with the moved anchor's lever arms)
    mv = lambda dz: [x + np.array([0, 0, dz]) if j in (2, 3) else x for j, x in enumerate(h)]
    for sgn in (1, -1):
        flip = sgn * bisect(lambda dz: oracle.probe_t3(og, mods, mv(sgn * dz)).passes(1), 0.0, 5.0)
        q, b, _ = oracle.probe_t3(og, mods, mv(flip)).cuts[1]
        assert abs(q - abs(res0 - (su + sv) * flip)) < 1e-4 * b and abs(q - b) < 1e-5 * b
        assert oracle.probe_t3(og, mods, mv(flip * 1.01)).failing() == [1]


@pytest.mark.parametrize("charge", [-1, 1])
def test_t3_curvature_cut(charge, full, og):
    """T3 curvature (Section 2.3): |kappa| of the circle through the three anchors may exceed the
    threshold curvature (x 1.01) by what the anchors' r-phi half pitches do to it, and no more."""
    lam, phi = 0.2, 0.3
    kap = -charge * 1.01 * KM * (1 - 1e-6)
    h, mods = _md_hits(full, phi, 0.0, 0.0, kap, lam, [0, 1, 2])
    A, B, C = h[0], h[2], h[4]
    p = oracle.probe_t3(og, mods, h)
    assert p.ok
    assert abs(p.cuts[0][0] - abs(curvature(f32(A), f32(B), f32(C)))) < 2e-6 * KM + 1e-4 * abs(kap)
    assert abs(p.attr[0] - curvature(f32(A), f32(B), f32(C))) < 1e-4 * abs(kap)
    n = _sagitta_dir(A, B, C)
    # the half pitches displace the anchors tangentially (about perpendicular to the chord):
    # the middle one away from the chord, the ends toward the other side
    sig = HP[0]
    Ae, Be, Ce = A - sig * n, B + sig * n, C - sig * n
    k_edge = abs(curvature(Ae, Be, Ce))
    def shifted(d):
        hh = list(h)
        hh[2], hh[3] = h[2] + d * n, h[3] + d * n
        return hh
    flip = bisect(lambda d: oracle.probe_t3(og, mods, shifted(d)).passes(0), 0.0, 1.0)
    k_flip = abs(curvature(A, B + flip * n, C))
    dk_phys = k_edge - abs(curvature(A, B, C))
    assert abs((k_flip - 1.01 * KM) - dk_phys) <= 0.05 * dk_phys
    assert dk_phys > 0.2 * (0.01 * KM)       # the error term dominates the 1% allowance


def _line_chi2(s, z, w):
    """chi2 of the weighted straight-line fit z = a + b s (numpy least squares)."""
    sw = np.sqrt(w)
    A = np.stack([np.ones_like(s), s], 1) * sw[:, None]
    coef, *_ = np.linalg.lstsq(A, z * sw, rcond=None)
    r = z * sw - A.dot(coef)
    return float(r.dot(r))


def _arc(points, kap):
    """Cumulative transverse arc lengths along a circle of curvature kap through the points."""
    s = [0.0]
    for a, b in zip(points[:-1], points[1:]):
        L = math.hypot(b[0] - a[0], b[1] - a[1])
        s.append(s[-1] + (2 * math.asin(abs(kap) * L / 2) / abs(kap) if kap else L))
    return np.array(s)


def test_t3_rz_chi2_cut(full, og_wide):
    """T3 r-z chi2 (Section 2.3): the weighted straight-line fit of z against the transverse arc
    length over the three anchors (errors: the half pitch along the strip) equals numpy's, and the
    cut falls at chi2 = 10."""
    lam, phi = 0.4, 0.3
    h, mods = _md_hits(full, phi, 0.0, 1.0, -K_CURV / 2.0, lam, [0, 1, 2])
    sig = np.array([HL[int(full.type[m])] for m in mods])

    def moved(dz):
        hh = list(h)
        hh[2], hh[3] = h[2] + np.array([0, 0, dz]), h[3] + np.array([0, 0, dz])
        return hh

    for dz in (0.0, 0.1, 0.3, -0.25):
        hh = moved(dz)
        P = [f32(hh[0]), f32(hh[2]), f32(hh[4])]
        kap = curvature(*P)
        chi2 = _line_chi2(_arc(P, kap), np.array([x[2] for x in P]), 1 / sig ** 2)
        pr = oracle.probe_t3(og_wide, mods, hh)
        assert len(pr.cuts) == 5 and pr.passes(1)
        assert abs(pr.cuts[4][0] - chi2) <= 2e-3 * chi2 + 1e-3
        assert pr.cuts[4][1] == 10.0
    flip = bisect(lambda dz: oracle.probe_t3(og_wide, mods, moved(dz)).passes(4), 0.0, 3.0)
    P = [f32(h[0]), f32(h[2]), f32(h[4])]
    s = _arc(P, curvature(*P))
    z = np.array([x[2] for x in P])
    # numpy's own flip: chi2 is quadratic in the displacement of one point
    c1 = _line_chi2(s, z + np.array([0, 1.0, 0]), 1 / sig ** 2)
    assert abs(flip - math.sqrt(10.0 / c1)) < 2e-3 * flip


# ----------------------------------------------------------------------- T5
def _t5_table():
    import json
    import os
    rec = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "t5_chi2_cuts.json")))
    xy = np.full(1024, rec["pooled"]["xy"])
    rz = np.full(1024, rec["pooled"]["rz"])
    for k, v in rec["categories"].items():
        if "xy" in v:
            xy[int(k)], rz[int(k)] = v["xy"], v["rz"]
    return xy, rz


def _category(g, mods):
    """sum_i kind_i 4^i over the anchors, innermost first; kind 0 barrel PS, 1 barrel 2S,
    2 endcap PS, 3 endcap 2S."""
    return sum(int(2 * g.subdet[m] + g.type[m]) * 4 ** i for i, m in enumerate(mods))


def _circle_chi2(P, sig):
    """chi2 of the quintuplet's circle model v = a + b u + c (u^2 + v^2) (frame: origin at the
    first point, u along the chord to the last, chord units; weights (chord / sigma)^2), by numpy
    least squares."""
    X = np.array([p[0] for p in P], np.float64)
    Y = np.array([p[1] for p in P], np.float64)
    ex, ey = X[-1] - X[0], Y[-1] - Y[0]
    L = math.hypot(ex, ey)
    ux, uy = ex / L, ey / L
    u = ((X - X[0]) * ux + (Y - Y[0]) * uy) / L
    v = ((Y - Y[0]) * ux - (X - X[0]) * uy) / L
    sw = L / np.asarray(sig)
    A = np.stack([np.ones_like(u), u, u * u + v * v], 1) * sw[:, None]
    coef, *_ = np.linalg.lstsq(A, v * sw, rcond=None)
    r = v * sw - A.dot(coef)
    return float(r.dot(r))


def test_t5_curvature_compatibility(full, og):
    """T5 radii (Section 2.3): |kappa_in - kappa_out| of the two triplets' circles is bounded by
    the sum of their curvature errors; moving the outer triplet's middle anchor away from its chord
    flips the cut where the circumcircle curvatures differ by that sum."""
    lam, phi = 0.3, 0.5
    h, mods = _md_hits(full, phi, 0.0, 0.0, -K_CURV / 3.0, lam, [0, 1, 2, 3, 4])
    p = oracle.probe_t5(og, mods, h)
    assert p.ok and all(p.extra)
    anchors = lambda hh: [f32(hh[2 * k]) for k in range(5)]
    a_in = oracle.probe_t3(og, mods[:3], h[:6]).attr
    a_out = oracle.probe_t3(og, mods[2:], h[4:]).attr
    assert abs(p.cuts[0][1] - (a_in[1] + a_out[1])) <= 1e-6 * p.cuts[0][1]
    A = anchors(h)
    n = _sagitta_dir(A[2], A[3], A[4])
    mv = lambda d: [x + d * n if j in (6, 7) else x for j, x in enumerate(h)]
    for d in (0.0, 0.002, -0.004):
        P = anchors(mv(d))
        dk = abs(curvature(P[0], P[1], P[2]) - curvature(P[2], P[3], P[4]))
        assert abs(oracle.probe_t5(og, mods, mv(d)).cuts[0][0] - dk) < 2e-3 * abs(a_in[0]) * 0.01 + 1e-7
    flip = bisect(lambda d: oracle.probe_t5(og, mods, mv(d)).passes(0), 0.0, 0.5)
    P = anchors(mv(flip))
    dk = abs(curvature(P[0], P[1], P[2]) - curvature(P[2], P[3], P[4]))
    assert abs(dk - p.cuts[0][1]) < 1e-3 * p.cuts[0][1]
    assert not oracle.probe_t5(og, mods, mv(flip * 1.01)).passes(0)


def test_t5_circle_chi2_cut_and_category(full, og_wide):
    """T5 circle fit (Section 2.3): chi2_xy equals numpy's least squares of the same model as the
    shared anchor moves off the circle, and the cut falls where that chi2 reaches the quintuplet's
    category cut (bPS bPS bPS b2S b2S here)."""
    xy, rz = _t5_table()
    lam, phi = 0.3, 0.5
    h, mods = _md_hits(full, phi, 0.0, 0.0, -K_CURV / 3.0, lam, [0, 1, 2, 3, 4])
    cat = _category(full, mods)
    assert cat == 320
    sig = [HP[int(full.type[m])] for m in mods]
    A = [f32(h[2 * k]) for k in range(5)]
    n = _sagitta_dir(A[0], A[2], A[4])
    mv = lambda d: [x + d * n if j in (4, 5) else x for j, x in enumerate(h)]
    for d in (0.0, 0.003, -0.006):
        pr = oracle.probe_t5(og_wide, mods, mv(d))
        assert pr.passes(0) and pr.passes(1)
        c2 = _circle_chi2([f32(mv(d)[2 * k]) for k in range(5)], sig)
        assert abs(pr.cuts[2][0] - c2) <= 3e-3 * c2 + 2e-3
        assert pr.cuts[2][1] == np.float32(xy[cat])
    flip = bisect(lambda d: oracle.probe_t5(og_wide, mods, mv(d)).passes(2), 0.0, 0.03)
    flip_np = bisect(lambda d: _circle_chi2([f32(mv(d)[2 * k]) for k in range(5)], sig) <= xy[cat], 0.0, 0.03)
    assert abs(flip - flip_np) <= 5e-3 * flip_np
    assert oracle.probe_t5(og_wide, mods, mv(flip)).passes(0)


def test_t5_rz_chi2_cut(full, og_wide):
    """T5 r-z line (Section 2.3): chi2_rz is numpy's weighted straight-line fit of z against the arc
    length (circle of the two triplets' mean curvature; errors: the half pitch along the strip),
    and the cut falls where it reaches the category's cut."""
    xy, rz = _t5_table()
    lam, phi = 0.3, 0.5
    h, mods = _md_hits(full, phi, 0.0, 0.0, -K_CURV / 3.0, lam, [0, 1, 2, 3, 4])
    cat = _category(full, mods)
    sig = np.array([HL[int(full.type[m])] for m in mods])
    mv = lambda dz: [x + np.array([0, 0, dz]) if j in (4, 5) else x for j, x in enumerate(h)]

    def chi2_np(hh):
        P = [f32(hh[2 * k]) for k in range(5)]
        kb = 0.5 * (curvature(P[0], P[1], P[2]) + curvature(P[2], P[3], P[4]))
        return _line_chi2(_arc(P, kb), np.array([x[2] for x in P]), 1 / sig ** 2)

    for dz in (0.0, 0.05, -0.09):
        pr = oracle.probe_t5(og_wide, mods, mv(dz))
        assert len(pr.cuts) == 8
        assert abs(pr.cuts[7][0] - chi2_np(mv(dz))) <= 2e-3 * pr.cuts[7][0] + 1e-4
        assert pr.cuts[7][1] == np.float32(rz[cat])
    flip = bisect(lambda dz: oracle.probe_t5(og_wide, mods, mv(dz)).passes(7), 0.0, 2.0)
    flip_np = bisect(lambda dz: chi2_np(mv(dz)) <= rz[cat], 0.0, 2.0)
    assert abs(flip - flip_np) <= 5e-3 * flip_np


def test_t5_cuts_follow_the_anchor_category(full, ofull):
    """Quintuplets of exact single tracks across |eta| < 2.4: each is tested against the cuts of
    its own category (ordered kinds of its anchors, innermost first)."""
    xy, rz = _t5_table()
    rng = np.random.Generator(np.random.PCG64(5))
    seen = set()
    for eta in np.linspace(-2.3, 2.3, 24):
        ev = make_single_track_event(full, 5.0, eta, rng.uniform(0, 2 * math.pi), z0=rng.uniform(-5, 5), q=1)
        r = oracle.run(ofull, ev, last=oracle.ST_T5)
        tup, _, _ = r.stage(oracle.ST_T5)
        for t in tup[:4]:
            mods = [int(ev.module[t[2 * k]]) for k in range(5)]
            hits = []
            for k in range(10):
                hits.append([ev.x[t[k]], ev.y[t[k]], ev.z[t[k]]])
            pr = oracle.probe_t5(ofull, mods, hits)
            assert pr.ok and len(pr.cuts) == 8
            c = _category(full, mods)
            assert pr.cuts[2][1] == np.float32(xy[c]) and pr.cuts[7][1] == np.float32(rz[c])
            seen.add(c)
    # barrel-only, barrel-endcap and endcap-only quintuplets, at least one not symmetric under
    # reversal of the anchor order
    kinds = lambda c: [c // 4 ** i % 4 for i in range(5)]
    assert len(seen) >= 5
    assert any(kinds(c) != kinds(c)[::-1] and xy[c] != xy[sum(k * 4 ** i for i, k in enumerate(kinds(c)[::-1]))]
               for c in seen)


# ------------------------------------------------------------------ pT3 / pT5
def _seeded(full, pt, eta, phi, q, layers, z0=0.5):
    """Exact pixel hits, exact seed (momentum at the innermost pixel hit) and outer MD hits of one
    helix; returns (pixel hits, MD hits, modules, seed, helix curvature)."""
    from lstgen.geometry import PIXEL_RADII
    kap = -q * K_CURV / pt
    lam = math.sinh(eta)
    pix = [at_r(phi, 0.0, z0, kap, lam, r) for r in PIXEL_RADII]
    s0 = cylinder_s(np.array([0.0]), np.array([kap]), PIXEL_RADII[0])[0]
    d = phi + kap * s0
    seed = (pt * math.cos(d), pt * math.sin(d), pt * lam, q)
    h, mods = _md_hits(full, phi, 0.0, z0, kap, lam, layers)
    return pix, h, mods, seed, kap


def _seed_circle(pix0, seed):
    """Centre and radius of the seed's circle: through the innermost pixel hit, tangent to the
    seed direction, curvature -q K / pT (counter-clockwise positive)."""
    px, py, _pz, q = seed
    pt = math.hypot(px, py)
    kap = -q * K_CURV / pt
    nx, ny = -py / pt, px / pt                      # left normal of the direction
    return np.array([pix0[0] + nx / kap, pix0[1] + ny / kap]), 1.0 / abs(kap), kap


def _dist_to_circle(p, c, R):
    return abs(math.hypot(p[0] - c[0], p[1] - c[1]) - R)


def _obj_attr(og, mods, h):
    a = oracle.probe_t3(og, mods[-3:] if len(mods) == 3 else mods[2:], h[-6:]).attr
    return float(a[0]), float(a[1])


def test_pt_window_at_first_anchor(full, og):
    """pT3/pT5 window (Section 2.4): the first anchor must lie within 1 cm of the seed's circle
    (measured across it) and, in z, within 3 cm plus two z errors of the seed's r-z line; and
    ahead of the pixel hit."""
    pix, h, mods, seed, kap = _seeded(full, 2.0, 0.3, 0.7, 1, [0, 1, 2])
    kT, dkT = _obj_attr(og, mods, h)
    c, R, _ = _seed_circle(f32(pix[0]), seed)
    p = oracle.probe_pt(og, mods, pix, h, seed, kT, dkT)
    assert p.ok, p.cuts
    assert p.cuts[0][2] == 1 and p.cuts[1][1] == 1.0
    assert p.cuts[1][0] < 1e-3 and abs(p.cuts[3][0]) < 2e-3
    mv = lambda a: [rot(x, a) if j < 2 else x for j, x in enumerate(h)]
    for sgn in (1, -1):
        flip = bisect(lambda a: oracle.probe_pt(og, mods, pix, mv(sgn * a), seed, kT, dkT).passes(1), 0.0, 0.2)
        A = f32(mv(sgn * flip)[0])
        assert abs(_dist_to_circle(A, c, R) - 1.0) < 0.02
        q1 = oracle.probe_pt(og, mods, pix, mv(sgn * flip * 0.5), seed, kT, dkT).cuts[1][0]
        assert abs(q1 - _dist_to_circle(f32(mv(sgn * flip * 0.5)[0]), c, R)) < 0.02 * q1
    # behind the pixel hit
    assert not oracle.probe_pt(og, mods, pix, mv(math.pi), seed, kT, dkT).passes(0)
    # z: 3 cm + 2 x the anchor's z error (half pitch along the strip, PS barrel)
    b = p.cuts[3][1]
    assert abs(b - (3.0 + 2 * HL[int(full.type[mods[0]])])) < 1e-6
    mz = lambda dz: [x + np.array([0, 0, dz]) if j < 2 else x for j, x in enumerate(h)]
    for sgn in (1, -1):
        flip = bisect(lambda dz: oracle.probe_pt(og, mods, pix, mz(sgn * dz), seed, kT, dkT).passes(3), 0.0, 10.0)
        assert abs(flip - b) < 3e-3


@pytest.mark.parametrize("k", [3, 5])
def test_pt_chi2_cuts(k, full, og):
    """pT3/pT5 chi2 (Section 2.4): the outer anchors are tested against the seed's own circle and
    r-z line, not refitted.  chi2_xy = sum of squared distances to the seed circle over the anchor
    error plus the seed's resolution carried to the anchor (2% curvature: the circle moves by
    dk d^2 / 2 at distance d; 1 mrad direction: by 1e-3 d); chi2_rz = sum of squared z residuals
    over the z errors.  Cuts 50 (pT3) and 80 (pT5)."""
    layers = [0, 1, 2] if k == 3 else [0, 1, 2, 3, 4]
    pix, h, mods, seed, kap = _seeded(full, 2.0, 0.3, 0.7, 1, layers)
    kT, dkT = _obj_attr(og, mods, h)
    c, R, ks = _seed_circle(f32(pix[0]), seed)
    X = 50.0 if k == 3 else 80.0
    ixy, irz, ik = 2 + k + 1, 2 + k + 2, 2 + k + 3
    p = oracle.probe_pt(og, mods, pix, h, seed, kT, dkT)
    assert p.ok and len(p.cuts) == ik + 1
    assert p.cuts[ixy][1] == X and p.cuts[irz][1] == X
    P0 = f32(pix[0])
    last = 2 * (k - 1)

    def seed_var(A, typ):
        d = math.hypot(A[0] - P0[0], A[1] - P0[1])
        c2, R2, _ = _seed_circle(P0, (seed[0] / 1.02, seed[1] / 1.02, seed[2], seed[3]))  # curvature +2%
        a = _dist_to_circle(A, c2, R2) - _dist_to_circle(A, c, R)
        th = 1e-3
        rs = (seed[0] * math.cos(th) - seed[1] * math.sin(th), seed[0] * math.sin(th) + seed[1] * math.cos(th),
              seed[2], seed[3])
        c3, R3, _ = _seed_circle(P0, rs)
        bb = _dist_to_circle(A, c3, R3) - _dist_to_circle(A, c, R)
        return HP[typ] ** 2 + a * a + bb * bb, d

    mv = lambda a: [rot(x, a) if j in (last, last + 1) else x for j, x in enumerate(h)]

    def chi2_cf(hh):
        tot = 0.0
        for i in range(k):
            A = f32(hh[2 * i])
            var, _ = seed_var(f32(h[2 * i]), int(full.type[mods[i]]))
            tot += _dist_to_circle(A, c, R) ** 2 / var
        return tot

    assert p.cuts[ixy][0] < 1e-3
    r_last = math.hypot(h[last][0], h[last][1])
    for dd in (0.6, -1.0, 1.5):           # tangential moves of the last anchor [cm]
        q = oracle.probe_pt(og, mods, pix, mv(dd / r_last), seed, kT, dkT).cuts[ixy][0]
        assert q > 0.5 and abs(q - chi2_cf(mv(dd / r_last))) <= 0.03 * q
    flip = bisect(lambda a: oracle.probe_pt(og, mods, pix, mv(a), seed, kT, dkT).passes(ixy), 0.0, 0.05)
    flip_cf = bisect(lambda a: chi2_cf(mv(a)) <= X, 0.0, 0.05)
    assert abs(flip - flip_cf) < 0.02 * flip_cf
    # r-z: the last anchor moved in z; the residual against the seed's line is the move itself
    sz = HL[int(full.type[mods[-1]])]
    mz = lambda dz: [x + np.array([0, 0, dz]) if j in (last, last + 1) else x for j, x in enumerate(h)]
    q0 = p.cuts[irz][0]
    assert q0 < 1e-2
    flip = bisect(lambda dz: oracle.probe_pt(og, mods, pix, mz(dz), seed, kT, dkT).passes(irz), 0.0, 30.0)
    assert abs(flip - math.sqrt(X - q0) * sz) < 3e-3 * flip + 1e-3


def test_pt_curvature_compatibility(full, og):
    """pT3/pT5 curvature (Section 2.4): the seed curvature may differ from the outer object's by
    three seed resolutions (2% each) plus the object's own curvature error."""
    pix, h, mods, seed, kap = _seeded(full, 2.0, 0.3, 0.7, -1, [0, 1, 2])
    kT, dkT = _obj_attr(og, mods, h)
    ks = float(np.float32(-seed[3] * K_CURV / math.hypot(np.float32(seed[0]), np.float32(seed[1]))))
    p = oracle.probe_pt(og, mods, pix, h, seed, kT, dkT)
    assert p.ok
    q, b, _ = p.cuts[-1]
    assert abs(q - abs(ks - kT)) < 1e-6 * abs(ks)
    assert abs(b - (3 * 0.02 * abs(ks) + dkT)) < 1e-6 * abs(ks)
    for sgn in (1, -1):
        edge = ks + sgn * (3 * 0.02 * abs(ks) + dkT)
        assert oracle.probe_pt(og, mods, pix, h, seed, edge - sgn * 1e-4 * abs(ks), dkT).passes(len(p.cuts) - 1)
        assert not oracle.probe_pt(og, mods, pix, h, seed, edge + sgn * 1e-4 * abs(ks), dkT).passes(len(p.cuts) - 1)


# ------------------------------------------------------- Section 2.5 cleaning
def _seeded_ev(g, pt, eta, phi, q, drop=()):
    ev = make_single_track_event(g, pt, eta, phi, z0=0.0, q=q, seeded=True)
    keep = np.ones(ev.n_hits, bool)
    outer = ev.module >= 0
    keep[outer] = ~np.isin(g.layer[ev.module[outer]], list(drop)) | (g.subdet[ev.module[outer]] != 0)
    new = np.cumsum(keep) - 1
    return Event(x=ev.x[keep], y=ev.y[keep], z=ev.z[keep], module=ev.module[keep], sensor=ev.sensor[keep],
                 sim=ev.sim[keep], px=ev.px, py=ev.py, pz=ev.pz, q=ev.q,
                 hits4=new[ev.hits4].astype(np.int32), seed_sim=ev.seed_sim)


def _merge(*evs):
    """One event holding the hits and seeds of several (seed hit indices shifted)."""
    off = np.cumsum([0] + [e.n_hits for e in evs])
    cat = lambda f: np.concatenate([getattr(e, f) for e in evs])
    h4 = np.concatenate([e.hits4.reshape(-1, 4) + o for e, o in zip(evs, off)]).astype(np.int32)
    return Event(x=cat("x"), y=cat("y"), z=cat("z"), module=cat("module"), sensor=cat("sensor"), sim=cat("sim"),
                 px=cat("px"), py=cat("py"), pz=cat("pz"), q=cat("q"), hits4=h4,
                 seed_sim=np.arange(len(h4), dtype=np.int32))


@pytest.mark.parametrize("dphi_b,expect", [(0.01, [0]), (0.2, [0, 2])])
def test_t5_near_a_pt5_is_cleaned(dphi_b, expect, barrel, obarrel):
    """Section 2.5: a surviving T5 whose direction is near (eta-phi) a pT5 candidate is not added."""
    a = _seeded_ev(barrel, 3.0, 0.1, 0.7, 1)
    b = make_single_track_event(barrel, 3.0, 0.1, 0.7 + dphi_b, q=1)
    r = oracle.run(obarrel, _merge(a, b))
    t5, k5, _ = r.stage(oracle.ST_T5)
    assert k5.sum() == 2                          # one surviving T5 per track
    _, f5, _ = r.stage(oracle.ST_PT5)
    assert f5.sum() == 1
    ty, _, _ = r.tc()
    assert sorted(ty.tolist()) == expect


@pytest.mark.parametrize("dphi_b,expect", [(0.01, [1]), (0.2, [1, 2])])
def test_t5_near_a_pt3_is_cleaned(dphi_b, expect, barrel, obarrel):
    """Section 2.5: a surviving T5 near a pT3 candidate is not added either."""
    a = _seeded_ev(barrel, 3.0, 0.1, 0.7, 1, drop=(5, 6))
    b = make_single_track_event(barrel, 3.0, 0.1, 0.7 + dphi_b, q=1)
    r = oracle.run(obarrel, _merge(a, b))
    _, k5, _ = r.stage(oracle.ST_T5)
    assert k5.sum() == 1
    assert r.count(oracle.ST_PT5) == 0
    ty, _, _ = r.tc()
    assert sorted(ty.tolist()) == expect


@pytest.mark.parametrize("dphi_b,expect", [(0.03, [0]), (0.3, [0, 3])])
def test_pls_near_a_candidate_is_cleaned(dphi_b, expect, barrel, obarrel):
    """Section 2.5: a pixel segment that no candidate uses still stays out when it is near one
    (distance 0.05 in eta-phi), and enters when it is far from all of them."""
    a = _seeded_ev(barrel, 3.0, 0.1, 0.7, 1)
    bare = _seeded_ev(barrel, 3.0, 0.1, 0.7 + dphi_b, 1, drop=(1, 2, 3, 4, 5, 6))
    r = oracle.run(obarrel, _merge(a, bare))
    _, fp, _ = r.stage(oracle.ST_PLS)
    assert fp.tolist() == [1, 1]                  # both survive the pLS duplicate removal
    ty, off, hits = r.tc()
    assert sorted(ty.tolist()) == expect


def _second_seed(ev, rot_ang, share_first):
    """A second seed on the same track: the same momentum, its pixel hits rotated by rot_ang
    (new hits), optionally sharing the first pixel hit itself."""
    h4 = ev.hits4[0]
    new = []
    for k in range(4):
        if k == 0 and share_first:
            continue
        p = rot(np.array([ev.x[h4[k]], ev.y[h4[k]], ev.z[h4[k]]], np.float64), rot_ang)
        new.append(p)
    n0 = ev.n_hits
    nh = len(new)
    x = np.concatenate([ev.x, np.array([p[0] for p in new], np.float32)])
    y = np.concatenate([ev.y, np.array([p[1] for p in new], np.float32)])
    z = np.concatenate([ev.z, np.array([p[2] for p in new], np.float32)])
    idx = list(range(n0, n0 + nh))
    h4b = ([int(h4[0])] + idx) if share_first else idx
    return Event(x=x, y=y, z=z, module=np.concatenate([ev.module, np.full(nh, -1, np.int32)]),
                 sensor=np.concatenate([ev.sensor, np.zeros(nh, np.int32)]),
                 sim=np.concatenate([ev.sim, np.zeros(nh, np.int32)]),
                 px=np.concatenate([ev.px, ev.px]), py=np.concatenate([ev.py, ev.py]),
                 pz=np.concatenate([ev.pz, ev.pz]), q=np.concatenate([ev.q, ev.q]),
                 hits4=np.array([list(h4), h4b], np.int32), seed_sim=np.array([0, 0], np.int32))


def _swap_seeds(ev):
    o = [1, 0]
    return Event(x=ev.x, y=ev.y, z=ev.z, module=ev.module, sensor=ev.sensor, sim=ev.sim, px=ev.px[o], py=ev.py[o],
                 pz=ev.pz[o], q=ev.q[o], hits4=ev.hits4[o], seed_sim=ev.seed_sim[o])


def test_two_seeds_on_one_t5_keep_the_better(barrel, obarrel):
    """Section 2.5, same-object rule: two distinct seeds (no shared pixel hit) that both make a
    pT5 with one T5 leave one pT5, the one with the smaller score, whichever seed comes first."""
    a = _seeded_ev(barrel, 3.0, 0.1, 0.7, 1)
    ev = _second_seed(a, 3e-4, share_first=False)
    kept = []
    for e in (ev, _swap_seeds(ev)):
        r = oracle.run(obarrel, e)
        t5, f5, a5 = r.stage(oracle.ST_PT5)
        assert len(t5) == 2 and np.array_equal(t5[0, 1:], t5[1, 1:])   # one outer object
        assert a5[0, 2] != a5[1, 2] and f5.sum() == 1
        assert f5[int(np.argmin(a5[:, 2]))] == 1
        _, fp, _ = r.stage(oracle.ST_PLS)
        assert fp.tolist() == [1, 1]                                   # not pLS duplicates
        ty, off, hits = r.tc()
        assert ty.tolist() == [0]
        kept.append(tuple(hits[:4]))
    assert kept[0] == kept[1]


def test_score_tie_is_broken_by_the_seed(barrel, obarrel):
    """Section 2.5 ranking: two seeds with the same first pixel hit and momentum give bit-identical
    pT5 scores on the same T5; the tie goes to the lower seed index, so swapping the seeds swaps
    which pixel hits the candidate carries."""
    a = _seeded_ev(barrel, 3.0, 0.1, 0.7, 1)
    ev = _second_seed(a, 3e-4, share_first=True)
    kept = []
    for e in (ev, _swap_seeds(ev)):
        r = oracle.run(obarrel, e)
        t5, f5, a5 = r.stage(oracle.ST_PT5)
        assert len(t5) == 2 and a5[0, 2] == a5[1, 2]
        assert f5.tolist() == [1, 0] and t5[0, 0] == 0
        ty, off, hits = r.tc()
        assert ty.tolist() == [0]
        kept.append(tuple(hits[:4]))
    assert kept[0] != kept[1] and kept[0] == tuple(ev.hits4[0]) and kept[1] == tuple(ev.hits4[1])


def test_near_rule_boundary(og):
    """Section 2.5 'near in eta-phi' (reading: same hemisphere and sin^2 dphi + dlam^2 / (1 +
    mean lam^2) < D^2): the boundary in azimuth at equal slope is sin(dphi) = D, in slope at equal
    azimuth dlam = D sqrt(1 + mean lam^2); opposite directions are never near."""
    D = 0.02
    for lam in (0.0, 1.5):
        for base in (0.3, 2.0):
            a = (math.cos(base), math.sin(base), lam)
            e = math.asin(D)
            b_in = (math.cos(base + e * 0.999), math.sin(base + e * 0.999), lam)
            b_out = (math.cos(base + e * 1.001), math.sin(base + e * 1.001), lam)
            assert oracle.probe_near(og, a, b_in, D) and not oracle.probe_near(og, a, b_out, D)
            # slope: mean slope lam + dl / 2
            f = lambda dl: dl * dl / (1 + (lam + dl / 2) ** 2) - D * D
            lo, hi = 0.0, 1.0
            for _ in range(80):
                mid = 0.5 * (lo + hi)
                lo, hi = (mid, hi) if f(mid) < 0 else (lo, mid)
            assert oracle.probe_near(og, a, (a[0] * 3, a[1] * 3, lam + lo * 0.999), D)
            assert not oracle.probe_near(og, a, (a[0], a[1], lam + lo * 1.001), D)
            assert not oracle.probe_near(og, a, (-a[0], -a[1], lam), D)


# ------------------------------------------------------------ seed-search order
def test_seed_search_pretest_drops_nothing(barrel, full):
    """The oracle's seed search skips (seed, object) pairs whose first anchor fails the window test
    widened by 1e-5 relative; testing every pair with the full predicate instead gives the same
    pT3 / pT5 objects, attributes, flags, track candidates and borderline lists."""
    from lstgen import make_event
    evs = [(barrel, make_event("tiny", 0)), (full, make_event("serve", 3, pu=40))]
    rng = np.random.default_rng(4)
    n = 40
    evs.append((barrel, make_single_track_event(barrel, np.exp(rng.uniform(np.log(0.8), np.log(20.0), n)),
                                                rng.uniform(-0.5, 0.5, n), rng.uniform(0, 2 * np.pi, n),
                                                z0=rng.normal(0, 5, n), q=np.where(rng.uniform(size=n) < 0.5, -1, 1),
                                                smear=True, seeded=True, seed=4, n_noise=50)))
    n_pt = 0
    for g, ev in evs:
        a, b = oracle.OracleGeometry(g), oracle.OracleGeometry(g)
        b.set_pt_plain(True)
        ra, rb = oracle.run(a, ev), oracle.run(b, ev)
        for st in (oracle.ST_PT3, oracle.ST_PT5):
            for x, y in zip(ra.stage(st), rb.stage(st)):
                assert np.array_equal(x, y)
            for x, y in zip(ra.border(st), rb.border(st)):
                assert np.array_equal(x, y)
            n_pt += ra.count(st)
        for x, y in zip(ra.tc(), rb.tc()):
            assert np.array_equal(x, y)
    assert n_pt > 1000


def test_dense_fixtures_reach_the_seed_search_regimes(barrel, obarrel):
    """The dense fixtures (tests/dense.py) hold seeds with 256-1,024 and more than 1,024 compatible
    triplets, and a seed with more than 16 pT5 (the per-seed caches and list of the HIP seed search);
    the oracle's counts, which the GPU parity test then compares object by object."""
    from dense import dense_event, spread_event
    r = oracle.run(obarrel, dense_event(barrel))
    n3 = np.bincount(r.stage(oracle.ST_PT3)[0][:, 0], minlength=3)
    assert n3[0] > 1024 and 256 < n3[1] <= 1024
    r = oracle.run(obarrel, spread_event(barrel))
    assert r.count(oracle.ST_PT5) > 16 and r.count(oracle.ST_PT3) > 1024
