"""Generator truth used by the closed-form checks (float64, from lstgen only)."""
import numpy as np

from lstgen.geometry import K_CURV, surface_crossing


def md_surfaces(geom, pt, eta, phi, z0=0.0, d0=0.0, q=1):
    """Surfaces a helix crosses, in crossing order, with the module of its mini-doublet there.

    Returns a list of (s, surface_key, module_or_-1): module is the common
    module of the lower- and upper-sensor crossings, -1 when the two crossings
    fall in different modules (a tile boundary between the sensors).
    """
    kappa = -q * K_CURV / pt
    lam = np.sinh(eta)
    arr = lambda v: np.array([float(v)])
    out = {}
    for surf in geom.surfaces():
        kind, idx, side, sensor, _pos = surf
        s, mod, *_ = surface_crossing(geom, surf, arr(phi), arr(d0), arr(z0), arr(kappa), arr(lam))
        key = (kind, idx, side)
        rec = out.setdefault(key, [None, None, None])
        if sensor == 0:
            rec[0] = float(s[0])
            rec[1] = int(mod[0])
        else:
            rec[2] = int(mod[0])
    res = []
    for key, (s, mlo, mup) in out.items():
        if s is None or not np.isfinite(s) or mlo is None or mlo < 0:
            continue
        res.append((s, key, mlo if (mup == mlo) else -1))
    res.sort()
    return res


def longest_md_run(crossings):
    """Length of the longest run of consecutive crossed surfaces that all hold an MD."""
    best = cur = 0
    for _s, _k, m in crossings:
        cur = cur + 1 if m >= 0 else 0
        best = max(best, cur)
    return best


def md_runs(crossings):
    """Lengths of all maximal runs of consecutive crossed surfaces holding an MD."""
    runs, cur = [], 0
    for _s, _k, m in crossings:
        if m >= 0:
            cur += 1
        else:
            if cur:
                runs.append(cur)
            cur = 0
    if cur:
        runs.append(cur)
    return runs


def kappa_true(pt, q):
    return -q * K_CURV / pt
