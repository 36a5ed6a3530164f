"""GPU parity of tile_sort (all schedules) against the CPU oracle, bit-exact."""
import numpy as np
import pytest

from paper_1507_01391_amd import inputs

pytestmark = pytest.mark.gpu

SMALL_SCHEDULES = ["bitonic", "thm2", "split", "naive"]


@pytest.fixture(scope="module")
def ts():
    import paper_1507_01391_amd as ts
    return ts


def run_and_compare(ts, oracle, keys, payload, off, schedule, max_len=None, f32=False):
    from tests.gpu_util import dev, host_i32, host_u32
    wk, wp, wperm = oracle.tile_sort(keys, payload, off, f32_ordered=f32, nthreads=8)
    k, p, perm = ts.tile_sort(dev(keys), None if payload is None else dev(payload), dev(off),
                              max_tile_len=max_len, f32_ordered=f32, schedule=schedule)
    ts.check_device_errors()
    assert np.array_equal(host_u32(k), wk.view(np.uint32))
    assert np.array_equal(host_i32(perm), wperm)
    if payload is not None:
        assert np.array_equal(host_u32(p).reshape(np.asarray(wp).shape), np.asarray(wp).view(np.uint32))


@pytest.mark.parametrize("schedule", SMALL_SCHEDULES)
def test_single_tile_4096(ts, oracle, schedule):
    keys, payload, off = inputs.single_tile(seed=1508)
    run_and_compare(ts, oracle, keys, payload, off, schedule)


@pytest.mark.parametrize("schedule", SMALL_SCHEDULES)
def test_batched_uneven_with_ties(ts, oracle, schedule):
    rng = np.random.default_rng(77)
    sizes = np.concatenate([[0, 1, 2, 63, 64, 65, 4095, 4096], rng.integers(0, 4097, size=40)])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    keys = rng.integers(0, 300, size=off[-1], dtype=np.uint32)       # many duplicates
    keys[::7] = rng.integers(0, 2**32, size=keys[::7].shape[0], dtype=np.uint32)
    payload = np.stack([np.arange(off[-1], dtype=np.uint32), rng.integers(0, 2**32, size=off[-1], dtype=np.uint32)])
    run_and_compare(ts, oracle, keys, payload, off, schedule, max_len=4096)


@pytest.mark.parametrize("schedule", SMALL_SCHEDULES)
def test_distributions(ts, oracle, schedule):
    rng = np.random.default_rng(5)
    tiles = []
    for kind in ("uniform", "zipf", "presorted", "reversed", "equal"):
        for _ in range(4):
            n = int(rng.integers(1, 4097))
            if kind == "uniform":
                k = rng.integers(0, 2**32, size=n, dtype=np.uint32)
            elif kind == "zipf":
                k = np.minimum(rng.zipf(1.2, size=n), 2**32 - 1).astype(np.uint32)
            elif kind == "presorted":
                k = np.sort(rng.integers(0, 2**32, size=n, dtype=np.uint32))
            elif kind == "reversed":
                k = np.sort(rng.integers(0, 2**32, size=n, dtype=np.uint32))[::-1].copy()
            else:
                k = np.full(n, 0xFFFFFFFF if rng.random() < 0.5 else 12345, np.uint32)
            tiles.append(k)
    off = np.concatenate([[0], np.cumsum([len(t) for t in tiles])]).astype(np.int64)
    keys = np.concatenate(tiles)
    run_and_compare(ts, oracle, keys, None, off, schedule, max_len=4096)


@pytest.mark.parametrize("schedule", SMALL_SCHEDULES)
def test_f32_keys_with_special_values(ts, oracle, schedule):
    rng = np.random.default_rng(3)
    x = rng.standard_normal(4096 * 3).astype(np.float32)
    x[:8] = np.array([-np.inf, np.inf, -0.0, 0.0, 1e-40, -1e-40, 3.0, -3.0], np.float32)
    rng.shuffle(x)
    off = np.arange(4, dtype=np.int64) * 4096
    payload = rng.uniform(-1, 1, size=x.shape[0]).astype(np.float32)
    run_and_compare(ts, oracle, x.view(np.uint32), payload.view(np.uint32), off, schedule, f32=True)


@pytest.mark.parametrize("schedule", ["split", "naive", "auto"])
@pytest.mark.parametrize("cap", [8192, 16384])
def test_large_tiles(ts, oracle, schedule, cap):
    rng = np.random.default_rng(cap)
    sizes = np.array([cap, cap - 1, 4097, 777, 0, cap])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    keys = rng.integers(0, 2**32, size=off[-1], dtype=np.uint32)
    keys[: off[-1] // 3] = rng.integers(0, 50, size=off[-1] // 3, dtype=np.uint32)
    payload = rng.integers(0, 2**32, size=off[-1], dtype=np.uint32)
    run_and_compare(ts, oracle, keys, payload, off, schedule, max_len=cap)


def test_segments_workload_sample(ts, oracle):
    keys, payload, off, _ = inputs.segments(seed=11, num_segments=60, hi=16384)
    run_and_compare(ts, oracle, keys, payload, off, "auto", max_len=16384)
