"""Oracle runs of many generated events in parallel processes (CPU only).

Each worker regenerates its event from (config, event number), runs the
serial oracle on it and returns a picklable snapshot of every stage, the
borderline lists and the track candidates, so that a test can compare many
full-size events with the HIP library without waiting for the oracle serially.
"""
import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import oracle

_GEOM = {}


class OracleSnapshot:
    """The parts of an oracle result that the parity helpers read."""

    def __init__(self, r):
        self._stage = {st: r.stage(st) for st in range(7)}
        self._border = {st: r.border(st) for st in range(7)}
        self._tc = r.tc()
        self._ext = r.extensions()

    def stage(self, st):
        return self._stage[st]

    def border(self, st):
        return self._border[st]

    def tc(self):
        return self._tc

    def extensions(self):
        return self._ext


def _run_one(spec):
    from lstgen import make_event
    from lstgen.events import geometry_for
    config, ev_no = spec
    if config not in _GEOM:
        _GEOM[config] = oracle.OracleGeometry(geometry_for(config))
    ev = make_event(config, ev_no)
    return ev, OracleSnapshot(oracle.run(_GEOM[config], ev))


def oracle_many(specs, workers=None):
    """(event, oracle snapshot) for [(config, event number), ...], in the order given."""
    n = workers or min(16, len(os.sched_getaffinity(0)), len(specs))
    with ProcessPoolExecutor(max_workers=max(1, n), mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_run_one, specs))
