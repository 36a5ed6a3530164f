"""GPU parity of tile_sort (all schedules) against the CPU oracle, bit-exact."""
import numpy as np
import pytest

from paper_1507_01391_amd import inputs

pytestmark = pytest.mark.gpu

SMALL_SCHEDULES = ["bitonic", "thm2", "split", "naive", "merge"]


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


@pytest.mark.parametrize("schedule", ["split", "naive", "auto", "merge", "thm2", "bitonic"])
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


# ---- merge schedule: tiles longer than one workgroup, packing of short tiles --------

EDGE_SIZES = [0, 1, 2, 63, 64, 65, 511, 512, 513, 1024, 1025, 2048, 2049, 4095, 4096, 4097,
              8191, 8192, 8193, 12289, 16384, 16385, 20000, 32767, 32768, 32769, 40000, 65536]


@pytest.mark.parametrize("pack,wide", [(1, 32768), (0, 32768), (1, 4096), (1, 8192), (0, 16384)])
def test_merge_edge_sizes(ts, oracle, pack, wide):
    """Tile lengths at every bin edge; with merge_wide = 4096 every tile above 4096 keys
    goes through pieces and merge rounds, with 32768 (the default) tiles up to 32768 keys
    are sorted whole by one workgroup and only the longer ones are merged."""
    rng = np.random.default_rng(21 + pack + wide)
    sizes = np.array(EDGE_SIZES)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    keys = rng.integers(0, 50, size=off[-1], dtype=np.uint32)           # heavy ties
    keys[::5] = rng.integers(0, 2**32, size=keys[::5].shape[0], dtype=np.uint32)
    payload = np.stack([np.arange(off[-1], dtype=np.uint32),
                        rng.integers(0, 2**32, size=off[-1], dtype=np.uint32)])
    prev, prev_w = ts.knob("merge_pack", 1), ts.knob("merge_wide", 32768)
    ts.tune("merge_pack", pack)
    ts.tune("merge_wide", wide)
    try:
        run_and_compare(ts, oracle, keys, payload, off, "merge", max_len=65536)
    finally:
        ts.tune("merge_pack", prev)
        ts.tune("merge_wide", prev_w)


@pytest.mark.parametrize("seed", [11, 12])
def test_merge_segments_workload_sample(ts, oracle, seed):
    keys, payload, off, kinds = inputs.segments(seed=seed, num_segments=300, hi=32768)
    assert set(kinds.tolist()) == set(range(len(inputs.SEGMENT_KINDS)))
    run_and_compare(ts, oracle, keys, payload, off, "auto", max_len=32768)


def test_merge_f32_keys_long_tiles(ts, oracle):
    rng = np.random.default_rng(31)
    sizes = [30000, 9000, 4096, 700, 32768]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = rng.standard_normal(off[-1]).astype(np.float32)
    x[:10] = np.array([-np.inf, np.inf, -0.0, 0.0, 1e-40, -1e-40, 3.0, -3.0, 0.0, -0.0], np.float32)
    x[40000:40010] = x[:10]
    pay = rng.uniform(-1, 1, size=off[-1]).astype(np.float32)
    run_and_compare(ts, oracle, x.view(np.uint32), pay.view(np.uint32), off, "merge",
                    max_len=32768, f32=True)


def test_merge_long_tile_up_to_limit(ts, oracle):
    rng = np.random.default_rng(41)
    sizes = [1 << 20, 100000, 3]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    keys = rng.integers(0, 2**32, size=off[-1], dtype=np.uint32)
    keys[:300000] = rng.integers(0, 1000, size=300000, dtype=np.uint32)
    run_and_compare(ts, oracle, keys, None, off, "merge", max_len=1 << 20)


def test_merge_more_tiles_than_one_binning_pass(ts, oracle):
    """1.1 million tiles of 0..5 keys: the binning kernel covers 1024 x 1024 tiles per
    pass, so this batch takes two passes of its tile loop."""
    rng = np.random.default_rng(123)
    sizes = rng.integers(0, 6, size=1_100_000)
    sizes[-3:] = [4096, 5000, 1]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    keys = rng.integers(0, 2**32, size=int(off[-1]), dtype=np.uint32)
    run_and_compare(ts, oracle, keys, None, off, "merge", max_len=8192)


def test_merge_skips_tiles_outside_the_arrays(ts):
    from tests.gpu_util import dev
    keys = np.arange(4000, dtype=np.uint32)[::-1].copy()
    off = np.array([0, 100, 5000], np.int64)             # tile 1 ends past the 4000 keys
    ts.tile_sort(dev(keys), None, dev(off), max_tile_len=8192, schedule="merge")
    with pytest.raises(RuntimeError, match="total_len"):
        ts.check_device_errors()


def test_merge_graph_replay(ts, oracle):
    """The launch sequence captured once (stream capture) and replayed: every replay,
    with eager work on the same buffers in between, equals the eager result."""
    import torch
    from tests.gpu_util import dev
    keys, payload, off, _ = inputs.segments(seed=13, num_segments=120, hi=32768)
    wk, wp, wperm = oracle.tile_sort(keys, payload, off, nthreads=8)
    d_k, d_p, d_o = dev(keys), dev(payload), dev(off)
    ko, po, pm = torch.empty_like(d_k), torch.empty_like(d_p), torch.empty(len(keys), dtype=torch.int32, device="cuda")

    def call():
        ts.tile_sort(d_k, d_p, d_o, max_tile_len=32768, schedule="merge", keys_out=ko,
                     payload_out=po, perm_out=pm)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        call()                                   # warm-up: workspace and launch caches
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    for rep in range(3):
        ko.fill_(0)
        pm.fill_(-1)
        po.fill_(7)
        ts.tile_sort(d_k, None, d_o, max_tile_len=32768, schedule="merge")   # eager work between
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(ko.cpu().numpy().view(np.uint32), wk.view(np.uint32)), rep
        assert np.array_equal(pm.cpu().numpy(), wperm), rep
        assert np.array_equal(po.cpu().numpy().view(np.uint32), np.asarray(wp).view(np.uint32)), rep
    ts.check_device_errors()


def test_merge_one_large_array(ts, oracle):
    """One array of 2^24 keys sorted as a single tile (pieces plus 12 merge rounds)."""
    rng = np.random.default_rng(43)
    n = 1 << 24
    keys = rng.integers(0, 2**32, size=n, dtype=np.uint32)
    keys[::3] = rng.integers(0, 4096, size=keys[::3].shape[0], dtype=np.uint32)   # ties
    payload = rng.integers(0, 2**32, size=n, dtype=np.uint32)
    off = np.array([0, n], np.int64)
    run_and_compare(ts, oracle, keys, payload, off, "merge", max_len=n)


@pytest.mark.parametrize("schedule", ["bitonic", "split", "merge", "naive"])
def test_64bit_payload(ts, oracle, schedule):
    """A float64 payload (two 32-bit words per element, elem_stride 2) follows the sort."""
    from tests.gpu_util import dev
    rng = np.random.default_rng(77)
    cap = 8192
    sizes = np.array([cap, 1, 0, 3000, cap - 1, 700])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(off[-1])
    keys = rng.integers(0, 1000, size=n, dtype=np.uint32)      # many ties
    pay = rng.standard_normal(n)                               # float64
    k, p, perm = ts.tile_sort(dev(keys), dev(pay), dev(off), max_tile_len=cap, schedule=schedule)
    ts.check_device_errors()
    wk, wp, wperm = oracle.tile_sort(keys, pay.view(np.uint32).reshape(n, 2).T.copy(), off)
    assert np.array_equal(k.cpu().numpy().view(np.uint32), wk)
    assert np.array_equal(perm.cpu().numpy(), wperm)
    assert np.array_equal(p.cpu().numpy().view(np.uint32).reshape(n, 2).T, wp)


@pytest.mark.parametrize("num_tiles", [3, 1024, 1100])
def test_split_payload_fused_and_routed(ts, oracle, num_tiles):
    """The split schedule gathers a small batch's payload in the sort kernel (up to
    sort_small_batch = 1024 tiles) and a larger batch's with the router; both agree with
    the oracle on a 3-channel planar payload."""
    from tests.gpu_util import dev
    rng = np.random.default_rng(num_tiles)
    sizes = rng.integers(0, 300, size=num_tiles)
    sizes[0] = 4096
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(off[-1])
    keys = rng.integers(0, 50, size=n, dtype=np.uint32)
    pay = rng.integers(0, 2**32, size=(3, n), dtype=np.uint32)
    k, p, perm = ts.tile_sort(dev(keys), dev(pay), dev(off), max_tile_len=4096, schedule="split")
    ts.check_device_errors()
    wk, wp, wperm = oracle.tile_sort(keys, pay, off, nthreads=8)
    assert np.array_equal(k.cpu().numpy().view(np.uint32), wk)
    assert np.array_equal(perm.cpu().numpy(), wperm)
    assert np.array_equal(p.cpu().numpy().view(np.uint32), wp)


# ---- Theorem 2 on 64 x 128 and 64 x 256 tiles (two and four wavefronts per tile) -----

@pytest.mark.parametrize("cap", [8192, 16384])
def test_thm2_wide_distributions(ts, oracle, cap):
    """Every key distribution of the segmented workload, ragged lengths around both
    capacities, two planar payload channels."""
    rng = np.random.default_rng(cap + 3)
    tiles = []
    for kind in ("uniform", "zipf", "presorted", "reversed", "equal", "binary"):
        for n in (cap, cap - 1, int(rng.integers(4097, cap)), int(rng.integers(1, 4097))):
            if kind == "uniform":
                k = rng.integers(0, 2**32, size=n, dtype=np.uint32)
            elif kind == "zipf":
                k = np.minimum(rng.zipf(1.2, size=n), 2**32 - 1).astype(np.uint32)
            elif kind == "presorted":
                k = np.sort(rng.integers(0, 2**32, size=n, dtype=np.uint32))
            elif kind == "reversed":
                k = np.sort(rng.integers(0, 2**32, size=n, dtype=np.uint32))[::-1].copy()
            elif kind == "equal":
                k = np.full(n, 0xFFFFFFFF if rng.random() < 0.5 else 12345, np.uint32)
            else:
                k = (rng.random(n) < 0.5).astype(np.uint32)
            tiles.append(k)
    off = np.concatenate([[0], np.cumsum([len(t) for t in tiles])]).astype(np.int64)
    keys = np.concatenate(tiles)
    payload = np.stack([np.arange(off[-1], dtype=np.uint32),
                        rng.integers(0, 2**32, size=off[-1], dtype=np.uint32)])
    run_and_compare(ts, oracle, keys, payload, off, "thm2", max_len=cap)


@pytest.mark.parametrize("schedule", ["thm2", "bitonic"])
@pytest.mark.parametrize("cap", [8192, 16384])
def test_thm2_wide_f32_and_edges(ts, oracle, cap, schedule):
    """fp32 keys with the special values and ragged lengths around the wavefront
    boundaries, on the schedules spread over 2 and 4 wavefronts."""
    rng = np.random.default_rng(cap + 4)
    sizes = [0, 1, 2, 63, 64, 65, 4095, 4096, 4097, cap // 2, cap - 64, cap - 1, cap]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = rng.standard_normal(int(off[-1])).astype(np.float32)
    x[:8] = np.array([-np.inf, np.inf, -0.0, 0.0, 1e-40, -1e-40, 3.0, -3.0], np.float32)
    x[8:10] = np.array([0x7FC00001, 0xFFC00002], np.uint32).view(np.float32)   # NaNs, by their bits
    rng.shuffle(x)
    payload = rng.integers(0, 2**32, size=int(off[-1]), dtype=np.uint32)
    run_and_compare(ts, oracle, x.view(np.uint32), payload, off, schedule, max_len=cap, f32=True)


# Keys at the edges of the range the sorting networks compare composites in, read as
# IEEE doubles: key 0 at position 0 is +0.0, keys below 2^22 give subnormal composites,
# 2^22 is the first normal one, and the top bit and all-ones keys give the largest.
EDGE_KEYS = np.array([0, 1, 2, 3, 2**21, 2**22 - 1, 2**22, 2**22 + 1, 2**30, 2**31 - 1, 2**31,
                      2**31 + 1, 0xFFFFFFFE, 0xFFFFFFFF], np.uint32)


@pytest.mark.parametrize("schedule,max_len", [("bitonic", 4096), ("thm2", 4096), ("bitonic", 16384),
                                              ("thm2", 16384), ("merge", 65536)])
def test_composite_range_edge_keys(ts, oracle, schedule, max_len):
    rng = np.random.default_rng(41)
    sizes = [s for s in (1, 2, 300, 1000, 4096, 4097, 9000, 16384, 20000, 32768, 40000) if s <= max_len]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    keys = rng.choice(EDGE_KEYS, size=int(off[-1]))
    payload = np.arange(off[-1], dtype=np.uint32)
    run_and_compare(ts, oracle, keys, payload, off, schedule, max_len=max_len)


def test_thm2_tile_longer_than_capacity_is_reported(ts):
    from tests.gpu_util import dev
    keys = np.zeros(16385, np.uint32)
    ts.tile_sort(dev(keys), None, dev(np.array([0, 16385], np.int64)), max_tile_len=16384,
                 schedule="thm2")
    with pytest.raises(RuntimeError, match="capacity"):
        ts.check_device_errors()
