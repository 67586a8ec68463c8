"""Synthetic outer-tracker geometry and its first-principles module map.

Detector model (a stand-in for the CMS Phase-2 outer tracker of Section 1):

* Barrel: six cylindrical layers at r = 23, 36, 51, 68, 89, 109 cm.  Each layer
  is tiled by bi-layer pT modules 10 cm long in r-phi and 5 cm long in z; the
  two sensors of a module are cylinders at r -/+ 0.13 cm (2.6 mm apart, inside
  the 2-4 mm spacing of Section 1).  Sector k of a layer covers
  phi in [2 pi k / n_phi, 2 pi (k+1) / n_phi) with n_phi = ceil(2 pi r / 10);
  z-ring j covers [-zmax + 5 j, -zmax + 5 (j+1)).
* Endcap: five disks per side at |z| = 131, 156, 185, 220, 265 cm, sensor planes
  at |z| -/+ 0.13 cm (the lower sensor is the one nearer the interaction
  point), 5 cm radial rings from r = 23 cm (the last ring is 108-110 cm), each
  ring split into ceil(2 pi r_mid / 10) phi sectors.
* Module type: PS (macro-pixel, 100 um x 1.5 mm) for the three inner barrel
  layers and endcap rings with r_mid < 60 cm; 2S (90 um strips, 5 cm long)
  elsewhere.
* Pixel seeding layers: cylinders at r = 3, 6.8, 10.9, 16 cm, |z| < 120 cm.

The module map (Section 2.2) lists, for every module, the modules of the next
surface outward that a helix crossing the module can reach, where the helix
has pT at or above the 0.8 GeV threshold and starts in the luminous region.
It is built by sweeping such helices through a grid of points on the module,
including its edges and corners, and adding a one-module margin around every
reached point.  The sweep uses the same closed-form helix propagation as the
event generator (``propagate``), all in float64.
"""
import hashlib
import math
import os
import tempfile

import numpy as np

# Magnetic field and the pT threshold (Section 2.2: 0.8 GeV).
B_TESLA = 3.8
K_CURV = 0.299792458 * B_TESLA / 100.0   # |kappa| [1/cm] = K_CURV / pT [GeV]
PT_MIN = 0.8
Z_LUM = 20.0          # half-length of the luminous region swept for the map [cm]
D0_MAX = 0.1          # transverse impact parameter covered by the map margin [cm]

SENSOR_HALF_GAP = 0.13
MOD_RPHI = 10.0
MOD_LONG = 5.0
BARREL_RADII = (23.0, 36.0, 51.0, 68.0, 89.0, 109.0)
DISK_Z = (131.0, 156.0, 185.0, 220.0, 265.0)
DISK_RMIN, DISK_RMAX = 23.0, 110.0
PIXEL_RADII = (3.0, 6.8, 10.9, 16.0)
PIXEL_ZMAX = 120.0

PS, TWO_S = 0, 1
BARREL, ENDCAP = 0, 1
# (r-phi pitch, long pitch) in cm for each module type.
PITCH = {PS: (0.010, 0.15), TWO_S: (0.009, 5.0)}

TWO_PI = 2.0 * math.pi


def _wrap_phi(phi):
    return np.mod(phi, TWO_PI)


class Geometry:
    """Module table (structure of arrays) plus lookup from surface points to modules.

    Module ids: barrel layers first (layer, z-ring, phi-sector), then endcap
    disks ordered (side -1 then +1, disk, ring, phi-sector).
    """

    def __init__(self, barrel_zmax, n_disks):
        self.barrel_zmax = float(barrel_zmax)
        self.n_disks = int(n_disks)
        self.n_zring = int(round(2 * barrel_zmax / MOD_LONG))
        self.layer_nphi = [int(math.ceil(TWO_PI * r / MOD_RPHI)) for r in BARREL_RADII]
        ring_lo = [DISK_RMIN + MOD_LONG * k for k in range(int(math.ceil((DISK_RMAX - DISK_RMIN) / MOD_LONG)))]
        self.ring_lo = np.array(ring_lo)
        self.ring_hi = np.minimum(self.ring_lo + MOD_LONG, DISK_RMAX)
        self.ring_nphi = [int(math.ceil(TWO_PI * 0.5 * (a + b) / MOD_RPHI))
                          for a, b in zip(self.ring_lo, self.ring_hi)]
        cols = {k: [] for k in ("subdet", "layer", "side", "type", "pos_lo", "pos_up",
                                "lmin", "lmax", "phimin", "phimax")}
        self.layer_base = []
        for li, r in enumerate(BARREL_RADII):
            self.layer_base.append(len(cols["subdet"]))
            nphi = self.layer_nphi[li]
            for j in range(self.n_zring):
                for k in range(nphi):
                    cols["subdet"].append(BARREL)
                    cols["layer"].append(li + 1)
                    cols["side"].append(0)
                    cols["type"].append(PS if li < 3 else TWO_S)
                    cols["pos_lo"].append(r - SENSOR_HALF_GAP)
                    cols["pos_up"].append(r + SENSOR_HALF_GAP)
                    cols["lmin"].append(-self.barrel_zmax + MOD_LONG * j)
                    cols["lmax"].append(-self.barrel_zmax + MOD_LONG * (j + 1))
                    cols["phimin"].append(TWO_PI * k / nphi)
                    cols["phimax"].append(TWO_PI * (k + 1) / nphi)
        self.ring_base = {}
        for side in (-1, 1):
            for d in range(self.n_disks):
                for ri in range(len(self.ring_lo)):
                    self.ring_base[(side, d, ri)] = len(cols["subdet"])
                    nphi = self.ring_nphi[ri]
                    rmid = 0.5 * (self.ring_lo[ri] + self.ring_hi[ri])
                    for k in range(nphi):
                        cols["subdet"].append(ENDCAP)
                        cols["layer"].append(d + 1)
                        cols["side"].append(side)
                        cols["type"].append(PS if rmid < 60.0 else TWO_S)
                        cols["pos_lo"].append(DISK_Z[d] - SENSOR_HALF_GAP)
                        cols["pos_up"].append(DISK_Z[d] + SENSOR_HALF_GAP)
                        cols["lmin"].append(self.ring_lo[ri])
                        cols["lmax"].append(self.ring_hi[ri])
                        cols["phimin"].append(TWO_PI * k / nphi)
                        cols["phimax"].append(TWO_PI * (k + 1) / nphi)
        self.subdet = np.array(cols["subdet"], np.int32)
        self.layer = np.array(cols["layer"], np.int32)
        self.side = np.array(cols["side"], np.int32)
        self.type = np.array(cols["type"], np.int32)
        self.pos_lo = np.array(cols["pos_lo"], np.float64)
        self.pos_up = np.array(cols["pos_up"], np.float64)
        self.lmin = np.array(cols["lmin"], np.float64)
        self.lmax = np.array(cols["lmax"], np.float64)
        self.phimin = np.array(cols["phimin"], np.float64)
        self.phimax = np.array(cols["phimax"], np.float64)
        self.n_modules = len(self.subdet)
        self.map_offsets = None
        self.map_targets = None

    # ------------------------------------------------------------------ surfaces
    def surfaces(self):
        """Every outer-tracker sensor surface: (kind, layer_or_disk, side, sensor, position).

        kind 'b': cylinder of radius `position`; kind 'e': plane at z = `position`
        (signed).  sensor 0 = lower, 1 = upper.
        """
        out = []
        for li, r in enumerate(BARREL_RADII):
            out.append(("b", li, 0, 0, r - SENSOR_HALF_GAP))
            out.append(("b", li, 0, 1, r + SENSOR_HALF_GAP))
        for side in (-1, 1):
            for d in range(self.n_disks):
                out.append(("e", d, side, 0, side * (DISK_Z[d] - SENSOR_HALF_GAP)))
                out.append(("e", d, side, 1, side * (DISK_Z[d] + SENSOR_HALF_GAP)))
        return out

    def lookup(self, kind, index, side, x, y, z):
        """Module id containing the point on the given surface, or -1 outside it."""
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        z = np.asarray(z, np.float64)
        phi = _wrap_phi(np.arctan2(y, x))
        out = np.full(x.shape, -1, np.int64)
        if kind == "b":
            nphi = self.layer_nphi[index]
            ring = np.floor((z + self.barrel_zmax) / MOD_LONG).astype(np.int64)
            ok = (z > -self.barrel_zmax) & (z < self.barrel_zmax) & (ring >= 0) & (ring < self.n_zring)
            sec = np.minimum(np.floor(phi / (TWO_PI / nphi)).astype(np.int64), nphi - 1)
            out[ok] = self.layer_base[index] + ring[ok] * nphi + sec[ok]
            return out
        rho = np.hypot(x, y)
        ok = (rho >= DISK_RMIN) & (rho < DISK_RMAX)
        ring = np.clip(np.floor((rho - DISK_RMIN) / MOD_LONG).astype(np.int64), 0, len(self.ring_lo) - 1)
        for ri in np.unique(ring[ok]):
            sel = ok & (ring == ri)
            nphi = self.ring_nphi[ri]
            sec = np.minimum(np.floor(phi[sel] / (TWO_PI / nphi)).astype(np.int64), nphi - 1)
            out[sel] = self.ring_base[(side, index, int(ri))] + sec
        return out

    def module_arrays(self):
        """Module description in the layout the library and oracle read (float32 positions)."""
        return dict(subdet=self.subdet, layer=self.layer, side=self.side, type=self.type,
                    pos_lo=self.pos_lo.astype(np.float32), pos_up=self.pos_up.astype(np.float32),
                    lmin=self.lmin.astype(np.float32), lmax=self.lmax.astype(np.float32))


# ---------------------------------------------------------------------- helices
def helix_point(phi0, d0, z0, kappa, lam, s):
    """Position after transverse arc length s of the helix with the given parameters.

    phi0: direction at the point of closest approach to the beam line, which is
    d0 * (-sin phi0, cos phi0); kappa = d(direction)/ds (positive: turns
    counter-clockwise); lam = dz/ds.
    """
    u = kappa * s
    px = np.sin(u) / kappa
    py = d0 + 2.0 * np.sin(0.5 * u) ** 2 / kappa
    c, sn = np.cos(phi0), np.sin(phi0)
    return c * px - sn * py, sn * px + c * py, z0 + lam * s


def cylinder_s(d0, kappa, r):
    """Arc length of the first crossing of radius r on the outgoing half-turn (nan if none)."""
    den = 2.0 * (1.0 + kappa * d0)
    X = kappa * kappa * (r * r - d0 * d0) / den
    ok = (X >= 0.0) & (X <= 2.0) & (r > np.abs(d0))
    half = np.arcsin(np.sqrt(np.clip(X, 0.0, 2.0) / 2.0))
    s = 2.0 * half / np.abs(kappa)
    return np.where(ok, s, np.nan)


def plane_s(z0, kappa, lam, zp):
    """Arc length of the crossing of plane z = zp on the outgoing half-turn (nan if none)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        s = (zp - z0) / lam
    ok = np.isfinite(s) & (s > 0.0) & (s <= math.pi / np.abs(kappa))
    return np.where(ok, s, np.nan)


def surface_crossing(geom, surf, phi0, d0, z0, kappa, lam):
    """(s, module, x, y, z) of the helices' crossing of one surface; module -1 if none."""
    kind, idx, side, _sensor, pos = surf
    if kind == "b":
        s = cylinder_s(d0, kappa, pos)
    else:
        s = plane_s(z0, kappa, lam, pos)
    sv = np.where(np.isfinite(s), s, 0.0)
    x, y, z = helix_point(phi0, d0, z0, kappa, lam, sv)
    mod = geom.lookup(kind, idx, side, x, y, z)
    mod = np.where(np.isfinite(s), mod, -1)
    return s, mod, x, y, z


def build_module_map(geom, n_pts_phi=5, n_pts_long=5, n_kappa=7, n_z0=3):
    """First-principles module map (Section 2.2) as CSR (offsets, targets).

    For each module, helices through an n_pts_phi x n_pts_long grid of points on
    its lower sensor (edges and corners included), with curvature sampled in
    [-kappa_max, kappa_max] (pT >= 0.8 GeV) and origin z0 sampled in
    [-Z_LUM, Z_LUM], are propagated to the next surface outward that they
    cross inside its active area.  The module reached there, and its
    neighbours one module away in phi and in the long coordinate, are targets.
    """
    kmax = K_CURV / PT_MIN
    lower = [s for s in geom.surfaces() if s[3] == 0]
    fp = np.linspace(0.0, 1.0, n_pts_phi)
    fl = np.linspace(0.0, 1.0, n_pts_long)
    kap = np.linspace(-kmax, kmax, n_kappa)
    kap = np.where(kap == 0.0, 1e-9, kap)
    z0s = np.linspace(-Z_LUM, Z_LUM, n_z0)
    FP, FL, KA, Z0 = np.meshgrid(fp, fl, kap, z0s, indexing="ij")
    FP, FL, KA, Z0 = FP.ravel(), FL.ravel(), KA.ravel(), Z0.ravel()
    per = FP.size
    src_all, dst_all = [], []
    chunk = 512
    for m0 in range(0, geom.n_modules, chunk):
        ms = np.arange(m0, min(m0 + chunk, geom.n_modules))
        M = np.repeat(ms, per)
        fp_, fl_, ka, z0 = (np.tile(a, ms.size) for a in (FP, FL, KA, Z0))
        phi = geom.phimin[M] + fp_ * (geom.phimax[M] - geom.phimin[M])
        lng = geom.lmin[M] + fl_ * (geom.lmax[M] - geom.lmin[M])
        barrel = geom.subdet[M] == BARREL
        rho = np.where(barrel, geom.pos_lo[M], lng)
        zp = np.where(barrel, lng, geom.side[M] * geom.pos_lo[M])
        # Helix from the origin (d0 = 0) through the point with curvature ka.
        a = np.clip(ka * rho / 2.0, -1.0, 1.0)
        phi0 = phi - np.arcsin(a)
        sp = 2.0 * np.arcsin(np.abs(a)) / np.abs(ka)
        lam = (zp - z0) / sp
        best_s = np.full(M.size, np.inf)
        best_x = np.zeros(M.size)
        best_y = np.zeros(M.size)
        best_z = np.zeros(M.size)
        best_surf = np.full(M.size, -1)
        for si, surf in enumerate(lower):
            s, mod, x, y, z = surface_crossing(geom, surf, phi0, 0.0, z0, ka, lam)
            take = (mod >= 0) & (s > sp + 0.2) & (s < best_s)
            best_s = np.where(take, s, best_s)
            best_x = np.where(take, x, best_x)
            best_y = np.where(take, y, best_y)
            best_z = np.where(take, z, best_z)
            best_surf = np.where(take, si, best_surf)
        for si, surf in enumerate(lower):
            sel = best_surf == si
            if not np.any(sel):
                continue
            kind, idx, side, _, pos = surf
            x, y, z = best_x[sel], best_y[sel], best_z[sel]
            rho_t = np.hypot(x, y)
            phi_t = np.arctan2(y, x)
            dphi = MOD_RPHI / rho_t
            for dp in (-1.0, 0.0, 1.0):
                for dl in (-1.0, 0.0, 1.0):
                    ph = phi_t + dp * dphi
                    if kind == "b":
                        xx, yy = rho_t * np.cos(ph), rho_t * np.sin(ph)
                        zz = z + dl * MOD_LONG
                    else:
                        rr = rho_t + dl * MOD_LONG
                        xx, yy = rr * np.cos(ph), rr * np.sin(ph)
                        zz = z
                    t = geom.lookup(kind, idx, side, xx, yy, zz)
                    ok = t >= 0
                    src_all.append(M[sel][ok])
                    dst_all.append(t[ok])
    src = np.concatenate(src_all)
    dst = np.concatenate(dst_all)
    pairs = np.unique(src.astype(np.int64) * geom.n_modules + dst.astype(np.int64))
    src = (pairs // geom.n_modules).astype(np.int64)
    dst = (pairs % geom.n_modules).astype(np.int32)
    offsets = np.zeros(geom.n_modules + 1, np.int64)
    np.add.at(offsets, src + 1, 1)
    offsets = np.cumsum(offsets).astype(np.int32)
    geom.map_offsets = offsets
    geom.map_targets = dst
    return offsets, dst


_CACHE = {}


def _cache_dir():
    d = os.environ.get("LSTGEN_CACHE") or os.path.join(tempfile.gettempdir(), "lstgen_cache")
    os.makedirs(d, exist_ok=True)
    return d


def _source_tag():
    with open(os.path.abspath(__file__), "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:16]


def _cached(key, make):
    """Geometry with its module map, memoised in-process and on disk (keyed by this file's hash)."""
    if key in _CACHE:
        return _CACHE[key]
    path = os.path.join(_cache_dir(), f"{key}_{_source_tag()}.npz")
    g = None
    if os.path.exists(path):
        try:
            with np.load(path) as z:
                g = make(build_map=False)
                g.map_offsets = z["off"]
                g.map_targets = z["tgt"]
        except Exception:
            g = None
    if g is None:
        g = make(build_map=True)
        tmp = path + f".{os.getpid()}.tmp.npz"
        np.savez(tmp, off=g.map_offsets, tgt=g.map_targets)
        os.replace(tmp, path)
    _CACHE[key] = g
    return g


def barrel_geometry():
    """Barrel-only detector, |z| < 60 cm, with its module map (5,736 modules)."""
    def make(build_map=True):
        g = Geometry(60.0, 0)
        if build_map:
            build_module_map(g)
        return g
    return _cached("barrel", make)


def full_geometry():
    """Barrel |z| < 120 cm plus 5 disks per side, with its module map (19,262 modules)."""
    def make(build_map=True):
        g = Geometry(120.0, len(DISK_Z))
        if build_map:
            build_module_map(g)
        return g
    return _cached("full", make)
