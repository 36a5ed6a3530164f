"""Seeded synthetic inputs for the five workloads.

This module only draws random numbers (numpy ``Generator(PCG64(seed))``) and
lays them out; it holds none of the sorting / partition / permutation
arithmetic, so both the HIP path and the CPU oracle can be fed from it.  The
paper (Afshani & Sitchinava) has no datasets or benchmarks; every workload is
synthetic with the shapes and value distributions stated below.

Workloads (sizes are the defaults; tests pass smaller ones):

* ``single_tile``   -- one tile of 4096 uint32 keys uniform in [0, 2^32) with
                       an index payload 0..4095.
* ``partition``     -- T tiles of n = 4096 uint32 labels holding exactly 64
                       copies of every value in [0, 64), shuffled per tile,
                       plus a one-channel float32 N(0,1) payload.
* ``permutation``   -- T tiles of n = 8192 float32 N(0,1) values with a
                       tile-local permutation pi: ``uniform`` (independent
                       shuffle per tile), ``transpose`` (the tile viewed as a
                       128 x 64 row-major matrix, pi(r*64+c) = c*128+r),
                       ``bitrev`` (13-bit bit reversal) or ``identity``.
* ``segments``      -- S segments with sizes floor(exp(U(ln 256, ln 32769)))
                       clipped to [256, 32768]; per segment keys are uniform
                       uint32, Zipf(1.2), presorted, reversed or all-equal;
                       payload is the index within the segment.
* ``sort_payload``  -- R rows of n = 16384 float32 N(0,1) keys (raw bits),
                       an 8-channel float32 U(-1,1) payload stored
                       channel-planar [C, R*n], and an upstream gradient
                       N(0,1) of the payload's shape.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 1507


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_offsets(num_tiles: int, n: int) -> np.ndarray:
    return np.arange(num_tiles + 1, dtype=np.int64) * n


def single_tile(seed: int = SEED_BASE + 1, n: int = 4096):
    rng = rng_for(seed)
    keys = rng.integers(0, 2**32, size=n, dtype=np.uint32)
    payload = np.arange(n, dtype=np.uint32)
    return keys, payload, uniform_offsets(1, n)


def partition(seed: int = SEED_BASE + 2, num_tiles: int = 65536, n: int = 4096,
              num_classes: int = 64):
    """Labels with exactly n / num_classes copies of each class per tile, shuffled per tile."""
    assert n % num_classes == 0
    rng = rng_for(seed)
    base = np.repeat(np.arange(num_classes, dtype=np.uint32), n // num_classes)
    labels = np.broadcast_to(base, (num_tiles, n))
    labels = rng.permuted(labels, axis=1).reshape(-1)
    payload = rng.standard_normal(num_tiles * n, dtype=np.float32)
    return labels, payload, uniform_offsets(num_tiles, n)


def random_labels(seed: int, num_tiles: int, n: int, num_classes: int):
    """Labels drawn independently and uniformly (unequal class sizes)."""
    rng = rng_for(seed)
    labels = rng.integers(0, num_classes, size=num_tiles * n, dtype=np.uint32)
    payload = rng.standard_normal(num_tiles * n, dtype=np.float32)
    return labels, payload, uniform_offsets(num_tiles, n)


def _bitrev(i: np.ndarray, bits: int) -> np.ndarray:
    out = np.zeros_like(i)
    for b in range(bits):
        out |= ((i >> b) & 1) << (bits - 1 - b)
    return out


def permutation_pi(family: str, n: int, num_tiles: int, rng: np.random.Generator) -> np.ndarray:
    if family == "uniform":
        base = np.broadcast_to(np.arange(n, dtype=np.int32), (num_tiles, n))
        return rng.permuted(base, axis=1).reshape(-1).astype(np.int32)
    if family == "identity":
        one = np.arange(n, dtype=np.int32)
    elif family == "transpose":
        assert n % 64 == 0
        rows = n // 64
        i = np.arange(n, dtype=np.int64)
        r, c = i // 64, i % 64
        one = (c * rows + r).astype(np.int32)
    elif family == "bitrev":
        bits = int(n).bit_length() - 1
        assert 1 << bits == n
        one = _bitrev(np.arange(n, dtype=np.int64), bits).astype(np.int32)
    else:
        raise ValueError(family)
    return np.tile(one, num_tiles)


def permutation(seed: int = SEED_BASE + 3, num_tiles: int = 16384, n: int = 8192,
                family: str = "uniform"):
    rng = rng_for(seed)
    x = rng.standard_normal(num_tiles * n, dtype=np.float32)
    pi = permutation_pi(family, n, num_tiles, rng)
    grad = rng.standard_normal(num_tiles * n, dtype=np.float32)
    return x, pi, grad, uniform_offsets(num_tiles, n)


SEGMENT_KINDS = ("uniform", "zipf", "presorted", "reversed", "equal")


def segment_sizes(rng: np.random.Generator, num_segments: int, lo: int = 256, hi: int = 32768):
    u = rng.uniform(np.log(lo), np.log(hi + 1), size=num_segments)
    return np.clip(np.floor(np.exp(u)).astype(np.int64), lo, hi)


def segments(seed: int = SEED_BASE + 4, num_segments: int = 100000, lo: int = 256,
             hi: int = 32768):
    rng = rng_for(seed)
    sizes = segment_sizes(rng, num_segments, lo, hi)
    offsets = np.zeros(num_segments + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    kinds = rng.integers(0, len(SEGMENT_KINDS), size=num_segments)
    total = int(offsets[-1])
    keys = np.empty(total, dtype=np.uint32)
    for s in range(num_segments):
        a, b = int(offsets[s]), int(offsets[s + 1])
        m = b - a
        kind = SEGMENT_KINDS[kinds[s]]
        if kind == "uniform":
            keys[a:b] = rng.integers(0, 2**32, size=m, dtype=np.uint32)
        elif kind == "zipf":
            z = rng.zipf(1.2, size=m)
            keys[a:b] = np.minimum(z, 2**32 - 1).astype(np.uint32)
        elif kind == "presorted":
            keys[a:b] = np.sort(rng.integers(0, 2**32, size=m, dtype=np.uint32))
        elif kind == "reversed":
            keys[a:b] = np.sort(rng.integers(0, 2**32, size=m, dtype=np.uint32))[::-1]
        else:
            keys[a:b] = np.uint32(rng.integers(0, 2**32, dtype=np.uint32))
    payload = (np.arange(total, dtype=np.int64) - np.repeat(offsets[:-1], sizes)).astype(np.uint32)
    return keys, payload, offsets, kinds


def sort_payload(seed: int = SEED_BASE + 5, rows: int = 4096, n: int = 16384, channels: int = 8):
    rng = rng_for(seed)
    keys = rng.standard_normal(rows * n, dtype=np.float32)
    payload = rng.uniform(-1.0, 1.0, size=(channels, rows * n)).astype(np.float32)
    grad = rng.standard_normal((channels, rows * n), dtype=np.float32)
    return keys, payload, grad, uniform_offsets(rows, n)
