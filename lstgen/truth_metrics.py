"""Physics performance of track candidates against generator truth.

Section 3 of the paper measures the track candidates with a hit-based match:
a candidate is matched to a simulated track when at least 75% of its hits
come from that track.  On the synthetic events the truth is the generator's
own: the track id of every hit, -1 for noise and for the hits of fake seeds.

* efficiency: fraction of the denominator tracks (pT above the threshold,
  |eta| inside the acceptance) that at least one candidate matches; also in
  bins of pT, of eta, of the transverse impact parameter and, for samples
  with displaced production vertices, of the vertex's transverse distance
  from the beam line (the paper's Delta_xy), as the paper plots it;
* fake rate: fraction of candidates matched to no track;
* duplicate rate: fraction of candidates whose track is matched by two or
  more candidates (all of them count, the first one too).

Each figure is also split by candidate type (pT5, pT3, T5, pLS), and the
efficiency by the type of the first candidate, in the order of the final
collection, that matches the track.  Nothing here is part of the
object-building chain: it reads the generator's truth and the chain's output.
"""
import numpy as np

TC_TYPES = ("pT5", "pT3", "T5", "pLS")
PT_BINS = (0.8, 0.9, 1.0, 1.5, 2.0, 5.0, 10.0, 50.0)
ETA_BINS = tuple(np.round(np.linspace(-2.4, 2.4, 13), 2))
D0_BINS = (0.0, 0.01, 0.02, 0.05, 0.5, 2.0, 5.0, 10.0)
DXY_BINS = (0.0, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.6)


def match_candidates(sim, offsets, hits, frac=0.75):
    """Matched track id of every candidate, -1 where no track owns `frac` of its hits."""
    out = np.full(len(offsets) - 1, -1, np.int64)
    for i in range(len(offsets) - 1):
        s = sim[hits[offsets[i]:offsets[i + 1]]]
        if s.size == 0:
            continue
        ids, cnt = np.unique(s, return_counts=True)
        k = int(np.argmax(cnt))
        if ids[k] >= 0 and cnt[k] >= frac * s.size:
            out[i] = ids[k]
    return out


def _binned(values, found, edges):
    """[(lo, hi, n, efficiency)] of `found` over the tracks whose value falls in each bin."""
    out = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (values >= lo) & (values < hi)
        n = int(sel.sum())
        out.append((float(lo), float(hi), n, float(found[sel].mean()) if n else None))
    return out


def tc_metrics(ev, types, offsets, hits, pt_min=0.9, eta_max=2.4, frac=0.75):
    """Efficiency, fake rate and duplicate rate of one event's track candidates.

    `types`, `offsets` and `hits` are the final collection as the chain
    returns it (type code 0..3 in TC_TYPES order, CSR offsets, event hit
    indices).  The efficiency denominator holds the tracks with pT > pt_min
    and |eta| < eta_max; the pT bins use the tracks with |eta| < eta_max
    only, so that the turn-on below pt_min is visible.
    """
    return pooled_metrics([(ev, (types, offsets, hits))], pt_min, eta_max, frac)


def pooled_metrics(events, pt_min=0.9, eta_max=2.4, frac=0.75):
    """The figures of tc_metrics over several events: [(event, (types, offsets, hits)), ...].

    Tracks and candidates of all events are pooled (a track of one event can
    only be matched by candidates of the same event).
    """
    types, matched, pt, eta, d0, dxy = [], [], [], [], [], []
    base = 0
    for ev, (ty, off, hits) in events:
        m = match_candidates(np.asarray(ev.sim), np.asarray(off), np.asarray(hits), frac)
        matched.append(np.where(m >= 0, m + base, -1))
        types.append(np.asarray(ty))
        pt.append(np.asarray(ev.tracks["pt"], np.float64))
        eta.append(np.asarray(ev.tracks["eta"], np.float64))
        d0.append(np.abs(np.asarray(ev.tracks["d0"], np.float64)))
        dxy.append(np.asarray(ev.tracks["dxy"], np.float64) if "dxy" in ev.tracks else np.full(pt[-1].size, np.nan))
        base += pt[-1].size
    types, matched = np.concatenate(types), np.concatenate(matched)
    pt, eta, d0, dxy = np.concatenate(pt), np.concatenate(eta), np.concatenate(d0), np.concatenate(dxy)

    n_match = np.bincount(matched[matched >= 0], minlength=pt.size)
    found_all = n_match > 0
    first_type = np.full(pt.size, -1)
    for i in range(len(matched) - 1, -1, -1):  # walking backwards leaves the first match
        if matched[i] >= 0:
            first_type[matched[i]] = types[i]
    in_eta = np.abs(eta) < eta_max
    denom = in_eta & (pt > pt_min)
    good = matched >= 0
    dup = np.zeros(len(matched), bool)
    dup[good] = n_match[matched[good]] > 1

    def rate(x, sel=None):
        x = x if sel is None else x[sel]
        return float(x.mean()) if x.size else 0.0

    out = {
        "events": len(events),
        "n_tc": int(len(matched)),
        "n_tracks": int(denom.sum()),
        "efficiency": rate(found_all[denom]),
        "fake_rate": rate(~good),
        "duplicate_rate": rate(dup),
        "by_type": {},
        "efficiency_vs_pt": _binned(pt[in_eta], found_all[in_eta], PT_BINS),
        "efficiency_vs_eta": _binned(eta[denom], found_all[denom], ETA_BINS),
        "efficiency_vs_d0": _binned(d0[denom], found_all[denom], D0_BINS),
    }
    if np.isfinite(dxy).any():
        # transverse distance of the production vertex from the beam line (displaced samples)
        out["efficiency_vs_dxy"] = _binned(dxy[denom], found_all[denom], DXY_BINS)
    for k, name in enumerate(TC_TYPES):
        sel = types == k
        out["by_type"][name] = {
            "n": int(sel.sum()),
            "fake_rate": rate(~good, sel),
            "duplicate_rate": rate(dup, sel),
            "efficiency": rate(first_type[denom] == k),
        }
    return out
