"""Calibrates the quintuplet chi2 cuts per category from the oracle alone.

Section 2.3 of the paper sets the quintuplet chi2 cuts empirically for each
category of quintuplets.  Category = the ordered kinds of the five anchors,
innermost first, kind = 2 * endcap + 2S (0 barrel PS, 1 barrel 2S, 2 endcap PS,
3 endcap 2S); index = sum_i kind_i 4^i.

Recipe: the oracle (no HIP code) runs to the quintuplet stage with both chi2
cuts opened on 20 PU200-like events of the `pu200` workload, generator events
900-919 (RNG seeds 2900-2919, disjoint from every event the tests and the
benchmark draw).  A quintuplet is truth-matched when its ten hits all belong to
one generated track of the primary sample (pT 0.8-50 GeV).  Per category with
at least MIN_ENTRIES truth-matched quintuplets, each cut is the 99.5% quantile
(the smallest observed value with at least 99.5% of the entries at or below it)
rounded up to three significant digits; every other category takes the same
quantile pooled over all categories.

Writes tests/golden/t5_chi2_cuts.json.  The oracle's and the HIP library's
frozen tables are typed from it; tests check both against it.

    python tests/golden/calibrate_t5_cuts.py [--workers N]
"""
import argparse
import json
import math
import multiprocessing as mp
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

QUANTILE = 0.995
MIN_ENTRIES = 50
EVENTS = list(range(900, 920))
CONFIG = "pu200"
OUT = os.path.join(HERE, "t5_chi2_cuts.json")

_OG = {}


def categories(geom, lower_hits, module):
    """Category index of each quintuplet from its five lower (anchor) hits."""
    m = module[lower_hits]                       # [n, 5]
    kind = 2 * geom.subdet[m] + geom.type[m]     # 0 barrel PS, 1 barrel 2S, 2 endcap PS, 3 endcap 2S
    return (kind * (4 ** np.arange(5))[None, :]).sum(1).astype(np.int64)


def _one(ev_no):
    import oracle
    from lstgen import make_event
    from lstgen.events import CONFIGS, geometry_for
    geom = geometry_for(CONFIG)
    if "og" not in _OG:
        og = oracle.OracleGeometry(geom)
        og.set_t5_cuts(np.full(1024, 1e30), np.full(1024, 1e30))
        _OG["og"] = og
    ev = make_event(CONFIG, ev_no)
    r = oracle.run(_OG["og"], ev, last=oracle.ST_T5)
    tup, _, attr = r.stage(oracle.ST_T5)
    sim = ev.sim[tup]                              # [n, 10]
    n_primary = CONFIGS[CONFIG]["n_trk"]
    matched = np.all(sim == sim[:, :1], axis=1) & (sim[:, 0] >= 0) & (sim[:, 0] < n_primary)
    cat = categories(geom, tup[:, 0::2], ev.module)
    return cat[matched], attr[matched, 1].astype(np.float64), attr[matched, 2].astype(np.float64), int(len(tup))


def quantile_up(v, q=QUANTILE):
    """Smallest observed value with a fraction >= q of the entries at or below it, rounded up to 3
    significant digits."""
    v = np.sort(np.asarray(v, np.float64))
    k = max(0, int(math.ceil(q * v.size)) - 1)
    x = float(v[k])
    if x <= 0:
        return 0.0
    e = math.floor(math.log10(x)) - 2
    return float(round(math.ceil(round(x / 10.0 ** e, 9)) * 10.0 ** e, 12))


def calibrate(workers):
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_one, EVENTS))
    cat = np.concatenate([p[0] for p in parts])
    xy = np.concatenate([p[1] for p in parts])
    rz = np.concatenate([p[2] for p in parts])
    out = {
        "recipe": {"config": CONFIG, "events": [EVENTS[0], EVENTS[-1]], "quantile": QUANTILE,
                   "min_entries": MIN_ENTRIES, "significant_digits": 3,
                   "truth": "all ten hits from one primary track (pT 0.8-50 GeV)"},
        "n_t5_all_open_cuts": int(sum(p[3] for p in parts)),
        "n_truth_matched": int(cat.size),
        "pooled": {"xy": quantile_up(xy), "rz": quantile_up(rz)},
        "categories": {},
    }
    for c in np.unique(cat):
        sel = cat == c
        n = int(sel.sum())
        kinds = [int(c) // 4 ** i % 4 for i in range(5)]
        rec = {"kinds": kinds, "n": n}
        if n >= MIN_ENTRIES:
            rec["xy"] = quantile_up(xy[sel])
            rec["rz"] = quantile_up(rz[sel])
        out["categories"][str(int(c))] = rec
    return out


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--workers", type=int, default=min(8, len(os.sched_getaffinity(0))))
    a = p.parse_args()
    res = calibrate(a.workers)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps({k: res[k] for k in ("n_t5_all_open_cuts", "n_truth_matched", "pooled")}))


if __name__ == "__main__":
    main()
