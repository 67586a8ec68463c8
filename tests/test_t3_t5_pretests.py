"""The triplet and quintuplet searches queue only the pairs that pass a pre-test
in fast arithmetic: for a triplet, the curvature cut and the azimuth-z test of
its three anchors (Section 2.3); for a quintuplet, the azimuth-z test of
anchors 1, 3 and 5.  Both must let through every object the exact selection
accepts.  This replays the pre-tests' formulas in IEEE float32 on the host
(the hardware reciprocal and reciprocal square root of the kernels taken
correctly rounded, 4 ulp high and 4 ulp low) and checks on a
PU200-like event that every triplet and quintuplet of the oracle passes them;
a dropped error term or a wrong factor rejects thousands of them.  It also
checks that the tests prune: of all (segment, segment) and (triplet, triplet)
pairs sharing an MD, few pass.
"""
import numpy as np
import pytest

import oracle
from lstgen.events import make_event, geometry_for

f32 = np.float32
K_CURV_D = 0.299792458 * 3.8 / 100.0
K_KMAX_CUT = f32(K_CURV_D / 0.8 * 1.01)
K_TAU = f32(0.8)
K_MARGIN, K_EPS = f32(1.001), f32(1e-6)
K_THIRD = f32(1.0 / 3.0)
D0 = f32(0.1)


@pytest.fixture(scope="module")
def objs():
    geom = geometry_for("pu200_seeded")
    ev = make_event("pu200_seeded", 5)
    r = oracle.run(oracle.OracleGeometry(geom), ev, last=3)
    md, _, _ = r.stage(0)
    ls, _, _ = r.stage(1)
    t3, _, _ = r.stage(2)
    t5, _, _ = r.stage(3)
    x, y, z = ev.x.astype(f32), ev.y.astype(f32), ev.z.astype(f32)
    endcap, is2s = geom.subdet == 1, geom.type == 1

    def anchors(hits):  # anchors = the lower hit of each MD (even positions of the hit tuple)
        h = hits[:, ::2]
        P = np.stack([x[h], y[h], z[h], np.sqrt(x[h] * x[h] + y[h] * y[h])], -1)
        m = ev.module[h]
        ec, t2 = endcap[m], is2s[m]
        hphi = np.where(t2, f32(0.0045), f32(0.005)).astype(f32)
        hlong = np.where(t2, f32(2.5), f32(0.075)).astype(f32)
        return P, dict(hphi=hphi, sig_t=np.where(ec, hphi + K_TAU * hlong, hphi).astype(f32),
                       ez=np.where(ec, f32(0), hlong).astype(f32))
    # candidates of the searches: every pair of objects where the outer MD of the first
    # is the inner MD of the second (two segments for a triplet, two triplets for a quintuplet)
    key = {(int(a), int(b)): i for i, (a, b) in enumerate(md)}
    seg = np.array([[key[(int(t[0]), int(t[1]))], key[(int(t[2]), int(t[3]))]] for t in ls])
    tri = np.array([[key[(int(t[0]), int(t[1]))], key[(int(t[4]), int(t[5]))]] for t in t3])

    def chained(first, last):
        order = np.argsort(first, kind="stable")
        cnt = np.bincount(first, minlength=len(md))
        off = np.concatenate([[0], np.cumsum(cnt)])
        ne = cnt[last]
        i = np.repeat(np.arange(len(last)), ne)
        j = order[np.repeat(off[last], ne) + np.arange(ne.sum()) - np.repeat(np.cumsum(ne) - ne, ne)]
        return i, j

    si, sj = chained(seg[:, 0], seg[:, 1])
    ti, tj = chained(tri[:, 0], tri[:, 1])
    lo = md[:, 0]
    cands = dict(t3=(anchors(np.stack([lo[seg[si, 0]], lo[seg[si, 1]], lo[seg[sj, 1]]], 1).repeat(2, 1)), len(t3)),
                 t5=(anchors(np.stack([lo[tri[ti, 0]], lo[tri[ti, 1]], lo[tri[tj, 1]]], 1).repeat(2, 1)), len(t5)))
    return anchors(t3), anchors(t5), cands


# The hardware reciprocal and reciprocal square root are within 1 ulp of the
# correctly rounded results; every replay runs with them exact and with each of them
# 4 ulp high, then 4 ulp low.
SCALES = (f32(1), f32(1 + 2.0 ** -21), f32(1 - 2.0 ** -21))


def rcp(x, sc):
    return (f32(1) / x) * sc


def rsq(x, sc):
    return (f32(1) / np.sqrt(x)) * sc


def phiz_may_pass(P, Q, R, mp, mq, mr, sc=SCALES[0]):
    su = (P[:, 0] * Q[:, 1] - P[:, 1] * Q[:, 0]) * rcp(P[:, 3] * Q[:, 3], sc)
    sv = (Q[:, 0] * R[:, 1] - Q[:, 1] * R[:, 0]) * rcp(Q[:, 3] * R[:, 3], sc)
    dzpq, dzqr = Q[:, 2] - P[:, 2], R[:, 2] - Q[:, 2]
    t1, t2 = su * dzqr, sv * dzpq
    iP, iQ, iR = rcp(P[:, 3], sc), rcp(Q[:, 3], sc), rcp(R[:, 3], sc)
    ePQ = (mp["hphi"] * iP + mq["hphi"] * iQ) + D0 * np.abs(iP - iQ)
    eQR = (mq["hphi"] * iQ + mr["hphi"] * iR) + D0 * np.abs(iQ - iR)
    au, av, adpq, adqr = np.abs(su), np.abs(sv), np.abs(dzpq), np.abs(dzqr)
    nl = (au * au + av * av) * K_THIRD
    tol = ((adqr * ePQ + adpq * eQR) + (au * (mq["ez"] + mr["ez"]) + av * (mp["ez"] + mq["ez"]))) + \
        nl * (au * adqr + av * adpq)
    return np.abs(t1 - t2) <= (tol * K_MARGIN + K_EPS) * f32(1.00001) + f32(1e-5) * (np.abs(t1) + np.abs(t2))


def curvature_may_pass(A, B, C, mA, mB, mC, sc=SCALES[0]):
    ux, uy = B[:, 0] - A[:, 0], B[:, 1] - A[:, 1]
    wx, wy = C[:, 0] - A[:, 0], C[:, 1] - A[:, 1]
    tx, ty = C[:, 0] - B[:, 0], C[:, 1] - B[:, 1]
    k = ux * wy - uy * wx
    lw2 = wx * wx + wy * wy
    kap = (f32(2) * k) * (rsq(ux * ux + uy * uy, sc) * rsq(lw2, sc) * rsq(tx * tx + ty * ty, sc))
    dk = (f32(4) * ((mA["sig_t"] + f32(2) * mB["sig_t"]) + mC["sig_t"])) * rcp(lw2, sc)
    return np.abs(kap) <= (K_KMAX_CUT + dk) * f32(1.00001)


def _pick(m, i):
    return {k: v[:, i] for k, v in m.items()}


@pytest.mark.parametrize("sc", SCALES)
def test_every_triplet_passes_its_pretest(objs, sc):
    (P, m), _, _ = objs
    assert len(P) > 50000
    A, B, C = P[:, 0], P[:, 1], P[:, 2]
    mA, mB, mC = _pick(m, 0), _pick(m, 1), _pick(m, 2)
    for name, ok in (("curvature", curvature_may_pass(A, B, C, mA, mB, mC, sc)),
                     ("azimuth-z", phiz_may_pass(A, B, C, mA, mB, mC, sc))):
        assert ok.all(), f"{name}: {np.count_nonzero(~ok)} of {len(ok)} triplets rejected"


@pytest.mark.parametrize("sc", SCALES)
def test_every_quintuplet_passes_its_pretest(objs, sc):
    _, (P, m), _ = objs
    assert len(P) > 5000
    ok = phiz_may_pass(P[:, 0], P[:, 2], P[:, 4], _pick(m, 0), _pick(m, 2), _pick(m, 4), sc)
    assert ok.all(), f"{np.count_nonzero(~ok)} of {len(ok)} quintuplets rejected"


def test_pretests_prune(objs):
    """The triplet pre-test keeps under 5% of the segment pairs, the quintuplet's azimuth-z
    test under half of the triplet pairs, and neither keeps fewer than the objects found."""
    _, _, cands = objs
    (P, m), n_t3 = cands["t3"]
    assert len(P) > 20 * n_t3
    A, B, C, mA, mB, mC = P[:, 0], P[:, 1], P[:, 2], _pick(m, 0), _pick(m, 1), _pick(m, 2)
    kept = np.count_nonzero(curvature_may_pass(A, B, C, mA, mB, mC) & phiz_may_pass(A, B, C, mA, mB, mC))
    assert n_t3 <= kept <= 0.05 * len(P), (kept, len(P), n_t3)
    (P, m), n_t5 = cands["t5"]
    kept = np.count_nonzero(phiz_may_pass(P[:, 0], P[:, 1], P[:, 2], _pick(m, 0), _pick(m, 1), _pick(m, 2)))
    assert n_t5 <= kept <= 0.5 * len(P), (kept, len(P), n_t5)
