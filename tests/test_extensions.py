"""Pins of the oracle's track extensions (Section 2.5, last part) to facts outside the oracle.

* closed form: for the exact hits of one helix, a candidate with outer MDs
  is lengthened by as many of the helix's later MDs as a chain of map-linked
  MDs from its last one reaches (at most two), its own hits kept in front;
* library routine: the circle fit over the 4 to 7 anchors of an extended
  chain equals numpy's weighted least squares, and its straight-line fit in
  (arc length, z) equals numpy's weighted polyfit over exact arc lengths;
* FP64 shadow: the extension decisions of the FP32 oracle and of its FP64
  build agree on small events.
"""
import math

import numpy as np
import pytest

import oracle
from lstgen import make_event, make_single_track_event

from test_oracle_pins import _tracks
from truth import md_surfaces

H_PHI = (0.005, 0.0045)
H_LONG = (0.075, 2.5)
TAU = 0.8


def _outer_pairs(ty, hits):
    """(lower, upper) hit pairs of a candidate's MDs, inner to outer."""
    h = hits[4:] if ty in (0, 1) else hits
    return [(int(h[2 * i]), int(h[2 * i + 1])) for i in range(len(h) // 2)]


@pytest.mark.parametrize("seeded", [False, True])
def test_single_track_extension_reaches_the_next_mds(seeded, full, ofull):
    pt, eta, phi, z0, q = _tracks(40, 61 + int(seeded), 2.4)
    off_map, tgt = full.map_offsets, full.map_targets
    n_ext = n_checked = 0
    for i in range(pt.size):
        ev = make_single_track_event(full, pt[i], eta[i], phi[i], z0=z0[i], q=q[i], seeded=seeded)
        r = oracle.run(ofull, ev)
        md_t, _, _ = r.stage(oracle.ST_MD)
        by_module = {}
        for lo, up in md_t:
            assert int(ev.module[lo]) not in by_module  # one MD per crossed module
            by_module[int(ev.module[lo])] = (int(lo), int(up))
        # the helix's MDs in crossing order; the module map may link an MD
        # to the next one or, over a crossing without an MD, to a later one
        seq = [by_module[m] for _s, _k, m in md_surfaces(full, pt[i], eta[i], phi[i], z0[i], 0.0, q[i])
               if m >= 0 and m in by_module]
        assert len(seq) == len(by_module)
        mod_of = {pr: int(ev.module[pr[0]]) for pr in seq}

        def linked(a, b):
            return seq.index(b) > seq.index(a) and mod_of[b] in tgt[off_map[mod_of[a]]:off_map[mod_of[a] + 1]]

        def succ(a):
            return [b for b in seq if linked(a, b)]

        ty, off, hits = r.tc()
        na, t3, _, xo, xh = r.extensions()
        for j in range(len(ty)):
            base = hits[off[j]:off[j + 1]]
            ext = xh[xo[j]:xo[j + 1]]
            assert np.array_equal(ext[:len(base)], base)
            if ty[j] == 3:
                assert na[j] == 0 and t3[j] == -1
                continue
            chain = _outer_pairs(ty[j], ext)
            assert all(linked(a, b) for a, b in zip(chain[:-1], chain[1:]))
            last = chain[len(chain) - na[j] - 1]
            # exact hits pass every cut, so the longest continuation (at most two MDs) is taken
            expect = 2 if any(succ(x) for x in succ(last)) else (1 if succ(last) else 0)
            assert na[j] == expect, (i, pt[i], eta[i], ty[j])
            n_checked += 1
            n_ext += expect > 0
    assert n_checked >= 30 and n_ext >= 8


def _sig_t(geom, m):
    ty = geom.type[m]
    return H_PHI[ty] + (TAU * H_LONG[ty] if geom.subdet[m] == 1 else 0.0)


def _sig_z(geom, m, lam):
    ty = geom.type[m]
    return H_LONG[ty] * abs(lam) + 0.01 if geom.subdet[m] == 1 else H_LONG[ty]


def _fits(geom, ev, lo):
    """(chi2_xy, chi2_rz, kappa) of the anchors `lo` by numpy, in float64."""
    X, Y, Z = (np.asarray(a, np.float64)[lo] for a in (ev.x, ev.y, ev.z))
    mods = np.asarray(ev.module)[lo]
    n = len(lo)
    ex, ey = X[-1] - X[0], Y[-1] - Y[0]
    L = math.hypot(ex, ey)
    ux, uy = ex / L, ey / L
    u = ((X - X[0]) * ux + (Y - Y[0]) * uy) / L
    v = ((Y - Y[0]) * ux - (X - X[0]) * uy) / L
    sw = np.array([L / _sig_t(geom, m) for m in mods])
    A = np.stack([np.ones(n), u, u * u + v * v], 1) * sw[:, None]
    coef, *_ = np.linalg.lstsq(A, v * sw, rcond=None)
    chi2xy = float(np.sum((v * sw - A.dot(coef)) ** 2))
    a, b, c = coef
    kap = 2 * c / (L * math.sqrt(1 + b * b - 4 * a * c))
    # exact arc lengths between consecutive anchors on the fitted circle
    Lc = np.hypot(np.diff(X), np.diff(Y))
    s = np.concatenate([[0.0], np.cumsum(2 * np.arcsin(kap * Lc / 2) / kap)])
    lam0 = (Z[-1] - Z[0]) / s[-1]
    w = np.array([1.0 / _sig_z(geom, m, lam0) for m in mods])
    line = np.polyfit(s, Z, 1, w=w)
    chi2rz = float(np.sum((w * (Z - np.polyval(line, s))) ** 2))
    return chi2xy, chi2rz, kap


def test_extension_fits_equal_numpy(full, ofull):
    og64 = oracle.OracleGeometry(full, f64=True)
    ev = make_event("pu200_seeded", 3)
    n_by_len = {}
    # FP32: the 3x3 normal equations of a 4-anchor chain lose ~1e-3 relative in
    # kappa and ~0.02 absolute in chi2 (against cuts of 10 and more); FP64 is exact
    for og, rtol, atol in ((ofull, 3e-3, 0.03), (og64, 1e-6, 1e-9)):
        r = oracle.run(og, ev)
        ty, off, hits = r.tc()
        na, _, at, xo, xh = r.extensions()
        sel = np.concatenate([np.nonzero((na > 0) & (ty == k))[0][:150] for k in range(3)])
        for j in sel:
            pairs = _outer_pairs(ty[j], xh[xo[j]:xo[j + 1]])
            lo = [p[0] for p in pairs]
            c2xy, c2rz, kap = _fits(full, ev, lo)
            assert abs(at[j, 2] - kap) <= rtol * abs(kap), (j, at[j], kap)
            assert abs(at[j, 0] - c2xy) <= rtol * c2xy + atol, (j, at[j], c2xy)
            assert abs(at[j, 1] - c2rz) <= rtol * c2rz + atol, (j, at[j], c2rz)
            n_by_len[len(lo)] = n_by_len.get(len(lo), 0) + 1
    assert all(n_by_len.get(n, 0) >= 10 for n in (4, 5, 6, 7)), n_by_len


def test_extension_fp64_shadow_agrees_on_small_events(barrel, obarrel):
    og64 = oracle.OracleGeometry(barrel, f64=True)
    n_ext = 0
    for k in range(4):
        ev = make_event("tiny", k)
        a, b = oracle.run(obarrel, ev), oracle.run(og64, ev)
        ea, eb = a.extensions(), b.extensions()
        assert np.array_equal(ea[0], eb[0]) and np.array_equal(ea[4], eb[4])
        n_ext += int((ea[0] > 0).sum())
    assert n_ext > 20
