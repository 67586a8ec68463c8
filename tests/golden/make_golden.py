"""Writes tests/golden/tiny_oracle.json from the oracle alone (no HIP code).

Per-stage object counts, duplicate-removal survivors and a digest of the track
candidates for the first five `tiny` events (barrel geometry, 100 helices,
200 noise hits; seeds 1000-1004).  Regenerate only when the oracle's
arithmetic changes, and name the passage that justifies the change in the
commit message.
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from lstgen import barrel_geometry, make_event  # noqa: E402


def digest(r):
    ty, off, hits = r.tc()
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(ty, np.int32).tobytes())
    h.update(np.ascontiguousarray(off, np.int32).tobytes())
    h.update(np.ascontiguousarray(hits, np.int32).tobytes())
    return h.hexdigest()


def compute():
    og = oracle.OracleGeometry(barrel_geometry())
    out = {}
    for ev_no in range(5):
        ev = make_event("tiny", ev_no)
        r = oracle.run(og, ev)
        out[str(ev_no)] = {
            "n_hits": ev.n_hits,
            "counts": [r.count(s) for s in range(8)],
            "t5_kept": int(r.stage(oracle.ST_T5)[1].sum()),
            "tc_digest": digest(r),
        }
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "tiny_oracle.json"), "w") as f:
        json.dump(compute(), f, indent=1, sort_keys=True)
        f.write("\n")
