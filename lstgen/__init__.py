"""Seeded synthetic inputs for the Line Segment Tracking chain.

This package draws detectors, module maps and events; it holds none of the
object-building arithmetic (no mini-doublet, segment, triplet, quintuplet or
cleaning selection).  Both the CPU oracle and the HIP library consume what it
writes, so it is the only code the two sides share.

The paper (arXiv:2207.08207) measures on a CMS ttbar + PU200 simulation in the
CMS Phase-2 outer tracker; neither is available, so these generators stand in
for them with the same shape: bi-layer pT modules (Section 1), a module map
built from first principles by sweeping helices above the pT threshold
(Section 2.2), PU200-like hit densities and pixel seeds (Section 2.4).
"""
from .geometry import Geometry, barrel_geometry, full_geometry
from .events import Event, make_event, make_single_track_event, CONFIGS

__all__ = ["Geometry", "barrel_geometry", "full_geometry", "Event",
           "make_event", "make_single_track_event", "CONFIGS"]
