"""The device-wide sort's reading of the partition-as-quicksort-step use (Sec. 1),
checked on the CPU with the oracle and numpy alone (no GPU code).

A pass of the device-wide sort partitions every 4096-key tile stably on one digit of
the key and stores tile t's block of digit d at goff[d][t], the exclusive prefix of the
per-tile digit counts taken in digit-major order.  These tests check the two facts the
sort rests on: one such pass is a stable partition of the whole array by the digit,
and six passes on digits of 6, 6, 6, 6, 6 and 2 bits (least significant first) are the
stable sort.
"""
import numpy as np
import pytest

TILE = 4096
DIGIT_BITS = [6, 6, 6, 6, 6, 2]


def one_pass(keys, payload, shift, nbits, oracle):
    """One pass as the device sort lays it out, with the oracle's per-tile partition."""
    n = keys.shape[0]
    T = (n + TILE - 1) // TILE
    digits = ((keys >> np.uint32(shift)) & np.uint32((1 << nbits) - 1)).astype(np.uint32)
    off = np.minimum(np.arange(T + 1, dtype=np.int64) * TILE, n)
    d_sorted, _, perm = oracle.tile_partition(digits, offsets=off, num_classes=64)
    hist = np.zeros((64, T), dtype=np.int64)
    for t in range(T):
        hist[:, t] = np.bincount(digits[off[t]:off[t + 1]], minlength=64)
    goff = (np.cumsum(hist.ravel()) - hist.ravel()).reshape(64, T)  # digit-major prefix
    out_k = np.empty_like(keys)
    out_p = np.empty_like(payload)
    for t in range(T):
        a, b = off[t], off[t + 1]
        src = a + perm[a:b]                      # tile items in partitioned order
        d = d_sorted[a:b].astype(np.int64)
        first = np.searchsorted(d, np.arange(64))  # where each digit's block starts in the tile
        dst = goff[d, t] + (np.arange(b - a) - first[d])
        out_k[dst] = keys[src]
        out_p[dst] = payload[src]
    return out_k, out_p


@pytest.mark.parametrize("n", [1, 4095, 4097, 3 * 4096 + 17])
def test_tiled_pass_is_a_global_stable_partition(oracle, n):
    rng = np.random.default_rng(n)
    keys = rng.integers(0, 2**32, size=n, dtype=np.uint32)
    idx = np.arange(n, dtype=np.uint32)
    for shift, nbits in ((0, 6), (12, 6), (30, 2)):
        k, p = one_pass(keys, idx, shift, nbits, oracle)
        digits = (keys >> np.uint32(shift)) & np.uint32((1 << nbits) - 1)
        want = np.argsort(digits, kind="stable")        # library stable partition
        assert np.array_equal(p, want.astype(np.uint32))
        assert np.array_equal(k, keys[want])


@pytest.mark.parametrize("dist", ["uniform", "few", "high_bits"])
def test_six_lsd_passes_are_the_stable_sort(oracle, dist):
    n = 2 * 4096 + 333
    rng = np.random.default_rng(7)
    if dist == "uniform":
        keys = rng.integers(0, 2**32, size=n, dtype=np.uint32)
    elif dist == "few":                                  # heavy ties
        keys = rng.integers(0, 5, size=n, dtype=np.uint32) * np.uint32(0x9E3779B1)
    else:                                                # only the last (2-bit) digit varies
        keys = rng.integers(0, 4, size=n, dtype=np.uint32) << np.uint32(30)
    k, p = keys.copy(), np.arange(n, dtype=np.uint32)
    shift = 0
    for nbits in DIGIT_BITS:
        k, p = one_pass(k, p, shift, nbits, oracle)
        shift += nbits
    assert shift == 32
    wk, _, wperm = oracle.tile_sort(keys)
    assert np.array_equal(k, wk)
    assert np.array_equal(p, wperm.astype(np.uint32))


def test_a_dropped_pass_is_seen(oracle):
    """Planted mistake: skipping the 2-bit top digit leaves the keys unsorted."""
    n = 4096 + 5
    keys = np.random.default_rng(3).integers(0, 2**32, size=n, dtype=np.uint32)
    k, p = keys.copy(), np.arange(n, dtype=np.uint32)
    shift = 0
    for nbits in DIGIT_BITS[:-1]:
        k, p = one_pass(k, p, shift, nbits, oracle)
        shift += nbits
    wk, _, _ = oracle.tile_sort(keys)
    assert not np.array_equal(k, wk)
