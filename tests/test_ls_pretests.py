"""The segment search's pre-tests (the module-level window bound, the candidate's
window, the inner MD's stub check and the pair pre-test before the exact
selection) must let through every segment the exact selection accepts.  The
kernels evaluate them with the hardware reciprocal and reciprocal square root
(within about 1 ulp of the correctly rounded operations) and margins of about
1e-4; this replays their formulas in IEEE float32 on the host, with those
operations correctly rounded, 4 ulp high and 4 ulp low, and checks on a
PU200-like event that every segment of the oracle passes all of them, so a
dropped term, a wrong sign or a margin on the wrong side fails here.  It also checks that the pair pre-test prunes: most pairs
past the first two tests fail it (Section 2.2's stub and window cuts).
"""
import numpy as np
import pytest

import oracle
from lstgen.events import make_event, geometry_for

f32 = np.float32
K_HALF_KMAX = f32(0.299792458 * 3.8 / 100.0 / 0.8 / 2.0)
K_MARGIN, K_EPS = f32(1.001), f32(1e-6)
D0 = f32(0.1)
# The hardware reciprocal and reciprocal square root are within 1 ulp of the
# correctly rounded results; the superset check runs with them exact and with each
# of them 4 ulp high, then 4 ulp low.
SCALES = (f32(1), f32(1 + 2.0 ** -21), f32(1 - 2.0 ** -21))


def rcp(x, sc):
    return (f32(1) / x) * sc


def rsq(x, sc):
    return (f32(1) / np.sqrt(x)) * sc


@pytest.fixture(scope="module")
def seg():
    geom = geometry_for("pu200_seeded")
    ev = make_event("pu200_seeded", 3)
    r = oracle.run(oracle.OracleGeometry(geom), ev, last=1)
    md, _, _ = r.stage(0)
    ls, _, _ = r.stage(1)
    x, y, z = ev.x.astype(f32), ev.y.astype(f32), ev.z.astype(f32)
    rr = np.sqrt(x * x + y * y)
    lo, up = md[:, 0], md[:, 1]
    A = np.stack([x[lo], y[lo], z[lo], rr[lo]], 1)
    mod = ev.module[lo].astype(np.int64)
    endcap = geom.subdet == 1
    is2s = geom.type == 1
    tau = (x[lo] * y[up] - y[lo] * x[up]) / rr[lo]
    dl = np.where(endcap[mod], np.abs(z[up]) - np.abs(z[lo]), rr[up] - rr[lo]).astype(f32)
    # anchor disc of each module: bounding box of its anchors
    M = geom.n_modules
    x0 = np.full(M, np.inf, f32); x1 = np.full(M, -np.inf, f32)
    y0 = np.full(M, np.inf, f32); y1 = np.full(M, -np.inf, f32)
    np.minimum.at(x0, mod, A[:, 0]); np.maximum.at(x1, mod, A[:, 0])
    np.minimum.at(y0, mod, A[:, 1]); np.maximum.at(y1, mod, A[:, 1])
    with np.errstate(invalid="ignore"):
        cx, cy = f32(0.5) * (x0 + x1), f32(0.5) * (y0 + y1)
        hx, hy = f32(0.5) * (x1 - x0), f32(0.5) * (y1 - y0)
        rho = np.sqrt(hx * hx + hy * hy) * f32(1.0001) + f32(1e-3)
        disc = np.stack([cx, cy, rho, np.sqrt(cx * cx + cy * cy)], 1).astype(f32)
    key = {(int(a), int(b)): i for i, (a, b) in enumerate(md)}
    la = np.array([key[(int(t[0]), int(t[1]))] for t in ls])
    lb = np.array([key[(int(t[2]), int(t[3]))] for t in ls])
    return dict(geom=geom, A=A, mod=mod, endcap=endcap, is2s=is2s, st=np.stack([tau, dl], 1).astype(f32),
                disc=disc, la=la, lb=lb, n_md=len(md))


def _info(s, m):
    ec, t2 = s["endcap"][m], s["is2s"][m]
    hphi = np.where(t2, f32(0.0045), f32(0.005)).astype(f32)
    hlong = np.where(t2, f32(2.5), f32(0.075)).astype(f32)
    er = np.where(ec, hlong, f32(0)).astype(f32)
    return ec, hphi, hlong, er


def window_bound(A, ma, disc, mb, s, sc=SCALES[0]):
    _, hphi_a, _, er_a = _info(s, ma)
    _, _, _, er_b = _info(s, mb)
    ub = K_HALF_KMAX * ((disc[:, 3] + disc[:, 2]) + er_b)
    ua = K_HALF_KMAX * (A[:, 3] - er_a)
    with np.errstate(invalid="ignore", divide="ignore"):
        w = (ub - ua) * rsq(f32(1) - ub * ub, sc) + (D0 + hphi_a + f32(0.005)) * rcp(A[:, 3], sc)
    return np.where(ub < f32(0.99), (w * K_MARGIN + K_EPS) * f32(1.01) + f32(1e-6), f32(3e38)).astype(f32)


def module_may_pass(A, disc, wm, sc=SCALES[0]):
    dn = np.abs(A[:, 0] * disc[:, 1] - A[:, 1] * disc[:, 0]) * rcp(A[:, 3], sc)
    return dn - disc[:, 2] <= (wm * (disc[:, 3] + disc[:, 2])) * f32(1.001) + f32(1e-4)


def window_may_pass(A, B, wm):
    return np.abs(A[:, 0] * B[:, 1] - A[:, 1] * B[:, 0]) <= wm * (A[:, 3] * B[:, 3])


def stub_may_pass(st, ec, hphi, sn, sx, sy, il, dz, eang, rp, sc):
    sn2 = sn * sn
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        pred_b = (st[:, 1] * sn) * rsq(f32(1) - sn2, sc)
        err_b = f32(2) * hphi + (f32(2) * st[:, 1]) * (eang + D0 * rcp(rp, sc))
        adz = np.abs(dz)
        ds = st[:, 1] * (sx * sx + sy * sy) * il * rcp(adz, sc)
        pred_e = ds * sn
        err_e = (f32(2) * hphi + f32(0.03) * np.abs(pred_e)) + ds * (eang + D0 * rcp(rp, sc))
    pred = np.where(ec, pred_e, pred_b)
    err = np.where(ec, err_e, err_b)
    ok = np.abs(st[:, 0] - pred) <= (err * K_MARGIN) * f32(1.0001) + K_EPS + f32(1e-4) * np.abs(pred)
    ok = np.where(~ec & ~(sn2 < f32(0.9)), True, ok)
    return np.where(ec & ~(adz > 0), False, ok)


def inner_stub_may_pass(A, B, sa, ma, mb, s, sc=SCALES[0]):
    ec_a, hphi_a, hlong_a, _ = _info(s, ma)
    ec_b, hphi_b, hlong_b, _ = _info(s, mb)
    sx, sy = B[:, 0] - A[:, 0], B[:, 1] - A[:, 1]
    il = rsq(sx * sx + sy * sy, sc)
    sn = (B[:, 0] * sy - B[:, 1] * sx) * rcp(B[:, 3], sc) * il
    eang = (np.where(ec_a, hlong_a, hphi_a) + np.where(ec_b, hlong_b, hphi_b)) * il
    return stub_may_pass(sa, ec_a, hphi_a, sn, sx, sy, il, B[:, 2] - A[:, 2], eang, A[:, 3], sc)


def pair_may_pass(A, B, sb, ma, mb, s, sc=SCALES[0]):
    ec_a, hphi_a, hlong_a, er_a = _info(s, ma)
    ec_b, hphi_b, hlong_b, er_b = _info(s, mb)
    dr = B[:, 3] - A[:, 3]
    ok = (dr > 0) & (A[:, 0] * B[:, 0] + A[:, 1] * B[:, 1] > 0)
    ub = K_HALF_KMAX * (B[:, 3] + er_b)
    ua = K_HALF_KMAX * (A[:, 3] - er_a)
    ra, rb = rcp(A[:, 3], sc), rcp(B[:, 3], sc)
    with np.errstate(invalid="ignore"):
        wv = (ub - ua) * rsq(f32(1) - ub * ub, sc) + (D0 * dr) * (ra * rb) + hphi_a * ra + hphi_b * rb
    c = A[:, 0] * B[:, 1] - A[:, 1] * B[:, 0]
    win = np.abs(c) <= ((wv * K_MARGIN + K_EPS) * (A[:, 3] * B[:, 3])) * f32(1.0001) + f32(1e-6)
    ok &= np.where(ub < f32(0.99), win, True)
    sx, sy = B[:, 0] - A[:, 0], B[:, 1] - A[:, 1]
    il = rsq(sx * sx + sy * sy, sc)
    sn = (A[:, 0] * sy - A[:, 1] * sx) * rcp(A[:, 3], sc) * il
    eang = (np.where(ec_a, hlong_a, hphi_a) + np.where(ec_b, hlong_b, hphi_b)) * il
    return ok & stub_may_pass(sb, ec_b, hphi_b, sn, sx, sy, il, B[:, 2] - A[:, 2], eang, B[:, 3], sc)


@pytest.mark.parametrize("sc", SCALES)
def test_every_segment_passes_every_pretest(seg, sc):
    s = seg
    a, b = s["la"], s["lb"]
    A, B = s["A"][a], s["A"][b]
    ma, mb = s["mod"][a], s["mod"][b]
    disc = s["disc"][mb]
    assert len(a) > 400000
    wm = window_bound(A, ma, disc, mb, s, sc)
    checks = {
        "module window bound": module_may_pass(A, disc, wm, sc),
        "candidate window": window_may_pass(A, B, wm),
        "inner stub": inner_stub_may_pass(A, B, s["st"][a], ma, mb, s, sc),
        "pair": pair_may_pass(A, B, s["st"][b], ma, mb, s, sc),
    }
    for name, ok in checks.items():
        assert ok.all(), f"{name}: {np.count_nonzero(~ok)} of {len(ok)} segments rejected"


def test_pair_pretest_prunes(seg):
    """On the candidates of a sample of inner MDs that pass the first two pre-tests, the
    pair pre-test keeps at most 40% and never fewer than the segments among them."""
    s = seg
    g = s["geom"]
    mo, mt = g.map_offsets.astype(np.int64), g.map_targets.astype(np.int64)
    md_off = np.searchsorted(s["mod"], np.arange(g.n_modules + 1))
    rng = np.random.default_rng(5)
    inner = np.sort(rng.choice(s["n_md"], 4000, replace=False))
    # every (inner MD, MD of a linked module) candidate of the sample
    ne = mo[s["mod"][inner] + 1] - mo[s["mod"][inner]]
    pair_a = np.repeat(inner, ne)
    tgt = mt[np.repeat(mo[s["mod"][inner]], ne) + np.arange(ne.sum()) - np.repeat(np.cumsum(ne) - ne, ne)]
    cnt = md_off[tgt + 1] - md_off[tgt]
    pa = np.repeat(pair_a, cnt)
    pb = np.repeat(md_off[tgt], cnt) + np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    A, B = s["A"][pa], s["A"][pb]
    ma, mb = s["mod"][pa], s["mod"][pb]
    disc = s["disc"][mb]
    wm = window_bound(A, ma, disc, mb, s)
    first = module_may_pass(A, disc, wm) & window_may_pass(A, B, wm) & inner_stub_may_pass(A, B, s["st"][pa], ma, mb, s)
    pair = first & pair_may_pass(A, B, s["st"][pb], ma, mb, s)
    segs = set(zip(s["la"].tolist(), s["lb"].tolist()))
    n_seg = sum((x, y) in segs for x, y in zip(pa[pair].tolist(), pb[pair].tolist()))
    n_seg_all = int(np.isin(s["la"], inner).sum())
    assert n_seg == n_seg_all
    assert first.sum() > 2 * n_seg_all
    assert pair.sum() <= 0.4 * first.sum(), (int(pair.sum()), int(first.sum()))
