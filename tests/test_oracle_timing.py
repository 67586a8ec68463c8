"""The oracle's own per-step wall clock, which the CPU baseline reports per stage."""
import time

import oracle
from lstgen import make_event


def test_step_seconds_cover_the_run(obarrel):
    ev = make_event("tiny", 0)
    t = time.perf_counter()
    r = oracle.run(obarrel, ev)
    wall = time.perf_counter() - t
    st = r.step_seconds()
    assert list(st) == oracle.STEP_NAMES
    assert all(v >= 0 for v in st.values()) and 0 < sum(st.values()) <= wall


def test_steps_not_reached_read_zero(obarrel):
    r = oracle.run(obarrel, make_event("tiny", 1), last=oracle.ST_LS)
    st = r.step_seconds()
    assert st["MD"] > 0 and st["LS"] > 0
    assert all(st[k] == 0.0 for k in oracle.STEP_NAMES[oracle.STEP_NAMES.index("T3"):])
