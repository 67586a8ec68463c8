"""Half-precision MD stubs (the paper's future work on half-precision types, Section 5).

* the oracle's rounding to binary16 (nearest, ties to even, subnormals,
  overflow) equals numpy's float32 -> float16 conversion bit for bit;
* on a PU200-like event the chain with binary16 stubs keeps the physics of
  the FP32 chain (efficiency, fake and duplicate rates within 0.002) and
  changes few segments.
"""
import numpy as np
import pytest

import oracle
from lstgen import make_event
from lstgen.truth_metrics import tc_metrics


def test_round_half_equals_numpy():
    lib = oracle._lib(False)
    rng = np.random.default_rng(3)
    v = np.concatenate([
        rng.uniform(-1, 1, 4000) * 10.0 ** rng.uniform(-9, 5, 4000),   # across the binades, subnormals included
        (np.arange(-2000, 2000) + 0.5) * 2.0 ** -24,                     # exact ties among subnormals
        (1024 + np.arange(0, 1000) + 0.5) * 2.0 ** -10,                  # exact ties in [1, 2)
        np.array([65504.0, 65519.0, 65520.0, 1e6, -1e6, 0.0, -0.0, 6.1e-5, 5.96e-8, 2.98e-8, 2.99e-8]),
    ]).astype(np.float32)
    got = np.array([lib.orc_round_half(float(x)) for x in v])
    with np.errstate(over="ignore"):
        want = v.astype(np.float16).astype(np.float64)
    same = (got == want) | (np.isnan(got) & np.isnan(want))
    assert same.all(), v[~same][:5]
    assert np.array_equal(np.signbit(got), np.signbit(want))


@pytest.mark.slow
def test_half_stubs_keep_the_physics(full):
    ev = make_event("pu200_seeded", 4)
    a = oracle.run(oracle.OracleGeometry(full), ev)
    b = oracle.run(oracle.OracleGeometry(full, stub16=True), ev)
    ma, mb = tc_metrics(ev, *a.tc()), tc_metrics(ev, *b.tc())
    for k in ("efficiency", "fake_rate", "duplicate_rate"):
        assert abs(ma[k] - mb[k]) < 0.002, (k, ma[k], mb[k])
    la, lb = a.count(oracle.ST_LS), b.count(oracle.ST_LS)
    assert abs(la - lb) < 0.01 * la
    print("LS", la, lb, "efficiency", ma["efficiency"], mb["efficiency"])
