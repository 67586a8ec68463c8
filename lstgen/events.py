"""Seeded synthetic events: closed-form helix hits, noise, pixel seeds.

Workloads (cm, GeV, B = 3.8 T):

* ``tiny``      barrel geometry (|z| < 60 cm); 100 helices with pT log-uniform in
                [0.8, 50], eta uniform in [-0.5, 0.5], phi uniform, z0 ~ N(0, 5),
                d0 ~ N(0, 0.01), charge +/-1; 200 uniform noise hits.
* ``pu200``     full geometry; 8,000 such helices with eta in [-2.4, 2.4] plus
                40,000 low-pT loopers (pT uniform in [0.1, 0.8]); noise hits
                make up 5% of the outer-tracker hits.
* ``pu200_seeded``  as ``pu200`` plus one pixel seed per track with pT > 0.8
                (four exact hits on the pixel cylinders, seed pT smeared by 2%,
                direction by 1 mrad, dz/ds exact) and 10% fake seeds.
* ``serve``     as ``pu200_seeded`` with pile-up PU ~ U[50, 250] (tracks and
                loopers scaled by PU / 200).
* ``batch``     as ``pu200_seeded`` with PU ~ U[140, 250].
* ``cube``      full geometry; 50 muons per event from production vertices
                uniform in a 5 cm cube centred on the origin (|x|, |y|, |z|
                <= 2.5 cm; transverse displacement up to 3.5 cm), pT
                log-uniform in [0.8, 50], eta uniform in [-2.4, 2.4]; 200
                noise hits; no pixel seeds.

Hits are the exact sensor crossings of ideal helices (no material, no
inefficiency), taken on the outgoing half-turn only, plus a uniform smear
within the pitch: the r-phi coordinate is rotated by U(-p/2, p/2) / r, the
long coordinate (z in the barrel, r in the endcap) is shifted by
U(-p_long/2, p_long/2).  The module is the one containing the exact crossing.
Hits are shuffled so that their order carries no track information.
Random numbers come from numpy's PCG64 seeded with 1000 * config + event.
"""
import math
from dataclasses import dataclass, field

import numpy as np

from .geometry import (BARREL, ENDCAP, K_CURV, PITCH, PIXEL_RADII, PIXEL_ZMAX,
                       TWO_PI, Geometry, barrel_geometry, cylinder_s, full_geometry,
                       helix_point, surface_crossing)

CONFIGS = {
    "tiny": dict(geom="barrel", n_trk=100, eta=0.5, n_loop=0, noise_abs=200, seeds=False),
    "pu200": dict(geom="full", n_trk=8000, eta=2.4, n_loop=40000, noise_frac=0.05, seeds=False),
    "pu200_seeded": dict(geom="full", n_trk=8000, eta=2.4, n_loop=40000, noise_frac=0.05, seeds=True),
    "serve": dict(geom="full", n_trk=8000, eta=2.4, n_loop=40000, noise_frac=0.05, seeds=True,
                  pu_range=(50.0, 250.0)),
    "batch": dict(geom="full", n_trk=8000, eta=2.4, n_loop=40000, noise_frac=0.05, seeds=True,
                  pu_range=(140.0, 250.0)),
    "cube": dict(geom="full", n_trk=50, eta=2.4, n_loop=0, noise_abs=200, seeds=False, cube=5.0),
}
CONFIG_NUMBER = {"tiny": 1, "pu200": 2, "pu200_seeded": 3, "serve": 4, "batch": 5, "cube": 6}


@dataclass
class Event:
    """One event in the layout both consumers read.

    Hits: x, y, z float32; module int32 (-1 for a pixel hit); sensor int32
    (0 lower, 1 upper).  Seeds: px, py, pz float32 at the innermost pixel hit,
    q int32, hits4 int32 [n_seeds, 4] (pixel-hit indices, innermost first).
    Truth: sim int32 per hit (-1 noise), seed_sim int32 per seed (-1 fake), and
    the per-track parameters.
    """
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    module: np.ndarray
    sensor: np.ndarray
    sim: np.ndarray
    px: np.ndarray = field(default_factory=lambda: np.zeros(0, np.float32))
    py: np.ndarray = field(default_factory=lambda: np.zeros(0, np.float32))
    pz: np.ndarray = field(default_factory=lambda: np.zeros(0, np.float32))
    q: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    hits4: np.ndarray = field(default_factory=lambda: np.zeros((0, 4), np.int32))
    seed_sim: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    tracks: dict = field(default_factory=dict)
    name: str = ""

    @property
    def n_hits(self):
        return int(self.x.size)

    @property
    def n_seeds(self):
        return int(self.px.size)


def _track_hits(geom, phi0, d0, z0, kappa, lam, smear, rng):
    """All outer-tracker hits of the given helices, as column arrays (float64)."""
    cols = {k: [] for k in ("x", "y", "z", "module", "sensor", "sim")}
    tid = np.arange(phi0.size)
    for surf in geom.surfaces():
        kind, _idx, _side, sensor, _pos = surf
        s, mod, x, y, z = surface_crossing(geom, surf, phi0, d0, z0, kappa, lam)
        ok = mod >= 0
        if not np.any(ok):
            continue
        x, y, z, mod = x[ok], y[ok], z[ok], mod[ok]
        if smear:
            ptype = geom.type[mod]
            p_rphi = np.where(ptype == 0, PITCH[0][0], PITCH[1][0])
            p_long = np.where(ptype == 0, PITCH[0][1], PITCH[1][1])
            rho = np.hypot(x, y)
            dphi = rng.uniform(-0.5, 0.5, x.size) * p_rphi / rho
            c, sn = np.cos(dphi), np.sin(dphi)
            x, y = c * x - sn * y, sn * x + c * y
            dl = rng.uniform(-0.5, 0.5, x.size) * p_long
            if kind == "b":
                z = z + dl
            else:
                f = (rho + dl) / rho
                x, y = x * f, y * f
        cols["x"].append(x)
        cols["y"].append(y)
        cols["z"].append(z)
        cols["module"].append(mod)
        cols["sensor"].append(np.full(x.size, sensor))
        cols["sim"].append(tid[ok])
    if not cols["x"]:
        return {k: np.zeros(0) for k in cols}
    return {k: np.concatenate(v) for k, v in cols.items()}


def _noise_hits(geom, n, rng):
    m = rng.integers(0, geom.n_modules, n)
    sensor = rng.integers(0, 2, n)
    phi = geom.phimin[m] + rng.uniform(0.0, 1.0, n) * (geom.phimax[m] - geom.phimin[m])
    lng = geom.lmin[m] + rng.uniform(0.0, 1.0, n) * (geom.lmax[m] - geom.lmin[m])
    pos = np.where(sensor == 0, geom.pos_lo[m], geom.pos_up[m])
    barrel = geom.subdet[m] == BARREL
    rho = np.where(barrel, pos, lng)
    z = np.where(barrel, lng, geom.side[m] * pos)
    return dict(x=rho * np.cos(phi), y=rho * np.sin(phi), z=z, module=m, sensor=sensor,
                sim=np.full(n, -1))


def _pixel_hits(phi0, d0, z0, kappa, lam):
    """Exact crossings of the four pixel cylinders; rows = tracks, nan where missed."""
    xs, ys, zs = [], [], []
    for r in PIXEL_RADII:
        s = cylinder_s(d0, kappa, r)
        x, y, z = helix_point(phi0, d0, z0, kappa, lam, np.where(np.isfinite(s), s, 0.0))
        bad = ~np.isfinite(s) | (np.abs(z) >= PIXEL_ZMAX)
        xs.append(np.where(bad, np.nan, x))
        ys.append(np.where(bad, np.nan, y))
        zs.append(np.where(bad, np.nan, z))
    return np.stack(xs, 1), np.stack(ys, 1), np.stack(zs, 1)


def _direction_at_inner_pixel(phi0, d0, kappa):
    s = cylinder_s(d0, kappa, PIXEL_RADII[0])
    return phi0 + kappa * s


def _draw_tracks(rng, n, eta_max, pt_lo, pt_hi, log_pt):
    if log_pt:
        pt = np.exp(rng.uniform(math.log(pt_lo), math.log(pt_hi), n))
    else:
        pt = rng.uniform(pt_lo, pt_hi, n)
    eta = rng.uniform(-eta_max, eta_max, n)
    phi = rng.uniform(0.0, TWO_PI, n)
    z0 = rng.normal(0.0, 5.0, n)
    d0 = rng.normal(0.0, 0.01, n)
    q = np.where(rng.uniform(0.0, 1.0, n) < 0.5, -1, 1)
    return dict(pt=pt, eta=eta, phi=phi, z0=z0, d0=d0, q=q)


def helix_from_vertex(vx, vy, vz, psi, kappa, lam):
    """(phi0, d0, z0, s_v) of the helix that passes the vertex (vx, vy, vz) with
    azimuthal direction psi there, in helix_point's parameters, and the arc
    length s_v of the vertex from the point of closest approach (negative:
    the vertex lies before it)."""
    rho = 1.0 / kappa
    cx = vx - rho * np.sin(psi)
    cy = vy + rho * np.cos(psi)
    D = np.hypot(cx, cy)
    sgn = np.sign(rho)
    # the centre is (d0 + rho) (-sin phi0, cos phi0); d0 + rho = sgn * D picks the near point
    phi0 = np.arctan2(-sgn * cx, sgn * cy)
    d0 = sgn * D - rho
    dpsi = np.mod(psi - phi0 + math.pi, TWO_PI) - math.pi
    s_v = dpsi / kappa
    return phi0, d0, vz - lam * s_v, s_v


def _draw_displaced(rng, n, eta_max, side):
    """Muons from vertices uniform in a cube of the given side centred on the origin."""
    pt = np.exp(rng.uniform(math.log(0.8), math.log(50.0), n))
    eta = rng.uniform(-eta_max, eta_max, n)
    psi = rng.uniform(0.0, TWO_PI, n)
    q = np.where(rng.uniform(0.0, 1.0, n) < 0.5, -1, 1)
    v = rng.uniform(-0.5 * side, 0.5 * side, (3, n))
    kappa = -q * K_CURV / pt
    phi0, d0, z0, _ = helix_from_vertex(v[0], v[1], v[2], psi, kappa, np.sinh(eta))
    return dict(pt=pt, eta=eta, phi=phi0, z0=z0, d0=d0, q=q, vx=v[0], vy=v[1], vz=v[2], psi=psi,
                dxy=np.hypot(v[0], v[1]))


def _assemble(geom, tracks, rng, smear, noise_abs=None, noise_frac=None, seeded=False,
              n_fake_seeds=None, fake_tracks=None, name=""):
    kappa = -tracks["q"] * K_CURV / tracks["pt"]
    lam = np.sinh(tracks["eta"])
    th = _track_hits(geom, tracks["phi"], tracks["d0"], tracks["z0"], kappa, lam, smear, rng)
    n_trk_hits = th["x"].size
    if noise_abs is not None:
        n_noise = int(noise_abs)
    elif noise_frac:
        n_noise = int(round(noise_frac / (1.0 - noise_frac) * n_trk_hits))
    else:
        n_noise = 0
    parts = [th]
    if n_noise:
        parts.append(_noise_hits(geom, n_noise, rng))
    outer = {k: np.concatenate([p[k] for p in parts]) for k in th}
    seeds = None
    pix = {k: np.zeros(0) for k in ("x", "y", "z", "sim")}
    if seeded:
        # One seed per track with pT > 0.8 GeV and all four pixel hits, plus fakes.
        sel = np.nonzero(tracks["pt"] > 0.8)[0]
        px_, py_, pz_ = _pixel_hits(tracks["phi"][sel], tracks["d0"][sel], tracks["z0"][sel],
                                    kappa[sel], lam[sel])
        good = np.all(np.isfinite(px_), axis=1)
        sel, px_, py_, pz_ = sel[good], px_[good], py_[good], pz_[good]
        n_true = sel.size
        n_fake = int(round(n_true / 9.0)) if n_fake_seeds is None else int(n_fake_seeds)
        if fake_tracks is None:
            fake_tracks = _draw_tracks(rng, n_fake, 2.4, 0.8, 50.0, True)
        fk = -fake_tracks["q"] * K_CURV / fake_tracks["pt"]
        fl = np.sinh(fake_tracks["eta"])
        fx, fy, fz = _pixel_hits(fake_tracks["phi"], fake_tracks["d0"], fake_tracks["z0"], fk, fl)
        fgood = np.all(np.isfinite(fx), axis=1)
        # Seed momentum at the innermost pixel hit: pT smeared by 2%, direction
        # rotated by 1 mrad, dz/ds kept exact.
        dirs = _direction_at_inner_pixel(tracks["phi"][sel], tracks["d0"][sel], kappa[sel])
        pt_s = tracks["pt"][sel] * (1.0 + 0.02 * rng.normal(0.0, 1.0, n_true))
        dirs = dirs + 0.001 * rng.normal(0.0, 1.0, n_true)
        fdir = _direction_at_inner_pixel(fake_tracks["phi"], fake_tracks["d0"], fk)
        seeds = dict(
            pt=np.concatenate([pt_s, fake_tracks["pt"][fgood]]),
            dirphi=np.concatenate([dirs, fdir[fgood]]),
            lam=np.concatenate([lam[sel], fl[fgood]]),
            q=np.concatenate([tracks["q"][sel], fake_tracks["q"][fgood]]),
            sim=np.concatenate([sel, np.full(int(fgood.sum()), -1)]),
            hx=np.concatenate([px_, fx[fgood]]), hy=np.concatenate([py_, fy[fgood]]),
            hz=np.concatenate([pz_, fz[fgood]]),
        )
        ns = seeds["pt"].size
        pix = dict(x=seeds["hx"].ravel(), y=seeds["hy"].ravel(), z=seeds["hz"].ravel(),
                   sim=np.repeat(seeds["sim"], 4))
    n_out = outer["x"].size
    n_pix = pix["x"].size
    n = n_out + n_pix
    perm = rng.permutation(n)          # new position of old hit k is inv[k]
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    x = np.concatenate([outer["x"], pix["x"]])[perm]
    y = np.concatenate([outer["y"], pix["y"]])[perm]
    z = np.concatenate([outer["z"], pix["z"]])[perm]
    module = np.concatenate([outer["module"], np.full(n_pix, -1)])[perm]
    sensor = np.concatenate([outer["sensor"], np.zeros(n_pix)])[perm]
    sim = np.concatenate([outer["sim"], pix["sim"]])[perm]
    ev = Event(x=x.astype(np.float32), y=y.astype(np.float32), z=z.astype(np.float32),
               module=module.astype(np.int32), sensor=sensor.astype(np.int32),
               sim=sim.astype(np.int32), tracks=tracks, name=name)
    if seeded and seeds["pt"].size:
        ns = seeds["pt"].size
        ev.px = (seeds["pt"] * np.cos(seeds["dirphi"])).astype(np.float32)
        ev.py = (seeds["pt"] * np.sin(seeds["dirphi"])).astype(np.float32)
        ev.pz = (seeds["pt"] * seeds["lam"]).astype(np.float32)
        ev.q = seeds["q"].astype(np.int32)
        ev.hits4 = inv[n_out + np.arange(4 * ns)].reshape(ns, 4).astype(np.int32)
        ev.seed_sim = seeds["sim"].astype(np.int32)
    return ev


def geometry_for(config):
    return barrel_geometry() if CONFIGS[config]["geom"] == "barrel" else full_geometry()


def make_event(config, event, pu=None, smear=True):
    """Event number `event` of a named workload (see module docstring)."""
    cfg = CONFIGS[config]
    geom = geometry_for(config)
    rng = np.random.Generator(np.random.PCG64(1000 * CONFIG_NUMBER[config] + int(event)))
    if pu is None and "pu_range" in cfg:
        pu = float(rng.uniform(*cfg["pu_range"]))
    scale = 1.0 if pu is None else pu / 200.0
    n_trk = int(round(cfg["n_trk"] * scale))
    n_loop = int(round(cfg["n_loop"] * scale))
    if "cube" in cfg:
        t1 = _draw_displaced(rng, n_trk, cfg["eta"], cfg["cube"])
    else:
        t1 = _draw_tracks(rng, n_trk, cfg["eta"], 0.8, 50.0, True)
    if n_loop:
        t2 = _draw_tracks(rng, n_loop, cfg["eta"], 0.1, 0.8, False)
        tracks = {k: np.concatenate([t1[k], t2[k]]) for k in t1}
    else:
        tracks = t1
    ev = _assemble(geom, tracks, rng, smear, noise_abs=cfg.get("noise_abs"),
                   noise_frac=cfg.get("noise_frac"), seeded=cfg["seeds"],
                   name=f"{config}#{event}")
    ev.tracks["pu"] = pu
    return ev


def make_single_track_event(geom, pt, eta, phi, z0=0.0, d0=0.0, q=1, smear=False,
                            seeded=False, seed=0, n_noise=0):
    """Event from explicitly given helices (scalars or arrays), for closed-form checks.

    With seeded=True every track with pT > 0.8 gets an unsmeared seed and no
    fake seed is added.
    """
    tr = dict(pt=np.atleast_1d(np.asarray(pt, np.float64)),
              eta=np.atleast_1d(np.asarray(eta, np.float64)),
              phi=np.atleast_1d(np.asarray(phi, np.float64)),
              z0=np.atleast_1d(np.asarray(z0, np.float64)),
              d0=np.atleast_1d(np.asarray(d0, np.float64)),
              q=np.atleast_1d(np.asarray(q, np.int64)))
    n = max(v.size for v in tr.values())
    tr = {k: np.broadcast_to(v, (n,)).copy() for k, v in tr.items()}
    rng = np.random.Generator(np.random.PCG64(seed))
    ev = _assemble(geom, tr, rng, smear, noise_abs=n_noise, seeded=seeded, n_fake_seeds=0,
                   fake_tracks=_draw_tracks(rng, 0, 2.4, 0.8, 50.0, True), name="explicit")
    if seeded and ev.n_seeds:
        # Unsmeared seeds: exact direction and pT at the innermost pixel hit.
        sel = ev.seed_sim
        kappa = -tr["q"][sel] * K_CURV / tr["pt"][sel]
        dirs = _direction_at_inner_pixel(tr["phi"][sel], tr["d0"][sel], kappa)
        lam = np.sinh(tr["eta"][sel])
        ev.px = (tr["pt"][sel] * np.cos(dirs)).astype(np.float32)
        ev.py = (tr["pt"][sel] * np.sin(dirs)).astype(np.float32)
        ev.pz = (tr["pt"][sel] * lam).astype(np.float32)
    return ev


def make_tiny_event(seed, n_tracks=10, n_noise=20, smear=True):
    """Small barrel event (<= n_tracks helices as in `tiny`, n_noise noise hits) for brute force."""
    geom = barrel_geometry()
    rng = np.random.Generator(np.random.PCG64(777000 + int(seed)))
    tracks = _draw_tracks(rng, n_tracks, 0.5, 0.8, 50.0, True)
    return _assemble(geom, tracks, rng, smear, noise_abs=n_noise, name=f"tinybf#{seed}")
