"""The sorting networks compare 64-bit composites (all below 2^62) with fp64 min and max.
This checks the IEEE-754 fact that makes that exact, on the host: bit patterns below 2^62
are non-negative, finite doubles (subnormal below 2^52) that order like the integers, and
min / max return an operand's bits unchanged."""
import numpy as np


def _composites(rng, n):
    parts = [rng.integers(0, 2**62, size=n, dtype=np.uint64),             # anywhere in range
             rng.integers(0, 2**52, size=n, dtype=np.uint64),             # subnormal doubles
             np.array([0, 1, 2**52 - 1, 2**52, 2**52 + 1, 2**62 - 2, 2**62 - 1], np.uint64)]
    return np.concatenate(parts)


def test_doubles_below_2_62_order_like_integers():
    rng = np.random.default_rng(3)
    c = _composites(rng, 20000)
    d = c.view(np.float64)
    assert np.all(np.isfinite(d)) and np.all(d >= 0) and not np.any(np.signbit(d))
    assert np.array_equal(np.argsort(c, kind="stable"), np.argsort(d, kind="stable"))


def test_min_max_return_operand_bits():
    rng = np.random.default_rng(4)
    a, b = _composites(rng, 5000), _composites(rng, 5000)[::-1].copy()
    lo = np.minimum(a.view(np.float64), b.view(np.float64)).view(np.uint64)
    hi = np.maximum(a.view(np.float64), b.view(np.float64)).view(np.uint64)
    assert np.array_equal(lo, np.minimum(a, b))
    assert np.array_equal(hi, np.maximum(a, b))


def test_complement_within_range_reverses_order():
    rng = np.random.default_rng(5)
    c = _composites(rng, 5000)
    mask = np.uint64(2**62 - 1)
    f = c ^ mask
    assert np.all(f <= mask)
    i, j = rng.integers(0, c.size, size=(2, 20000))
    assert np.array_equal(c[i] < c[j], f[i] > f[j])
