"""The MD kernels' pair index: quotient and remainder of t / n from a float
reciprocal with one correction step each way (divmod22 in the kernels).

IEEE single precision with round-to-nearest is the same on the host (numpy
float32) and in the kernels (v_mul_f32 and the correctly rounded division the
kernels are compiled with), so the host replays the kernel's arithmetic
exactly.  Below 2^22 the float quotient is within (t / n) 2^-23 < 1/2 of t / n,
so after truncation it is off by at most one, which the corrections undo; the
test checks that claim over every divisor the MD search meets (1..4,096 hits
per sensor) at the quotient boundaries, where rounding could go wrong, and on
a random sample.
"""
import numpy as np


def divmod22(t, n):
    t = np.asarray(t, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64)
    rn = np.float32(1.0) / n.astype(np.float32)
    q = (t.astype(np.float32) * rn).astype(np.int64)  # truncation of a non-negative float
    r = t - q * n
    low = r < 0
    q = np.where(low, q - 1, q)
    r = np.where(low, r + n, r)
    high = r >= n
    q = np.where(high, q + 1, q)
    r = np.where(high, r - n, r)
    return q, r


def test_exact_at_quotient_boundaries():
    limit = 1 << 22
    for n in range(1, 4097):
        k = np.arange(1, limit // n + 1, dtype=np.int64)
        t = np.concatenate([k * n - 1, k * n, k * n + 1])
        t = t[(t >= 0) & (t < limit)]
        q, r = divmod22(t, n)
        assert np.array_equal(q, t // n), n
        assert np.array_equal(r, t % n), n


def test_exact_on_random_pairs():
    rng = np.random.default_rng(22)
    n = rng.integers(1, 1 << 12, size=2_000_000)
    t = rng.integers(0, 1 << 22, size=n.size)
    q, r = divmod22(t, n)
    assert np.array_equal(q, t // n) and np.array_equal(r, t % n)


def test_a_plain_truncation_is_not_enough():
    # without the correction steps the float quotient is one off somewhere in the range
    t = np.arange(0, 1 << 22, dtype=np.int64)
    bad = 0
    for n in (3, 7, 11, 13, 97, 641, 1023):
        rn = np.float32(1.0) / np.float32(n)
        q = (t.astype(np.float32) * rn).astype(np.int64)
        bad += int(np.count_nonzero(q != t // n))
    assert bad > 0
