"""FP64 shadow report: how far the FP32 oracle's decisions and attributes
drift from the same selections evaluated in double precision.

TEST INFRASTRUCTURE ONLY (see the package docstring).  For each stage it
reports the objects only one precision builds (decision flips near a cut)
and, for the objects both build, the largest relative difference of each
attribute (chi2, curvature, ...), i.e. how much cut margin FP32 rounding
consumes.
"""
import numpy as np

from . import ATTR_W, ST_TC, STAGE_NAMES, OracleGeometry, run


def shadow_report(geom, ev, og32=None, og64=None):
    og32 = og32 or OracleGeometry(geom)
    og64 = og64 or OracleGeometry(geom, f64=True)
    a = run(og32, ev)
    b = run(og64, ev)
    rep = {}
    for st in range(ST_TC):
        ta, fa, aa = a.stage(st)
        tb, fb, ab = b.stage(st)
        ka = {tuple(t): i for i, t in enumerate(ta)}
        kb = {tuple(t): i for i, t in enumerate(tb)}
        common = [k for k in ka if k in kb]
        r = {"fp32": len(ka), "fp64": len(kb), "only_fp32": len(ka) - len(common),
             "only_fp64": len(kb) - len(common), "border_fp32": int(a.border(st)[0].shape[0]),
             "keep_flips": int(sum(int(fa[ka[k]]) != int(fb[kb[k]]) for k in common))}
        if ATTR_W[st] and common:
            ia = np.array([ka[k] for k in common])
            ib = np.array([kb[k] for k in common])
            x = aa[ia].astype(np.float64)
            y = ab[ib]
            rel = np.abs(x - y) / np.maximum(np.abs(y), 1e-30)
            r["max_rel_attr_drift"] = [float(v) for v in np.max(rel, axis=0)]
            r["median_rel_attr_drift"] = [float(v) for v in np.median(rel, axis=0)]
        rep[STAGE_NAMES[st]] = r
    ta, _, _ = a.tc()
    tb, _, _ = b.tc()
    rep["TC"] = {"fp32": int(ta.size), "fp64": int(tb.size)}
    return rep
