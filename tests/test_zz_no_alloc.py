"""tile_sort_noalloc (the entry point for callers that cannot allocate) against
tile_sort on the same inputs, through the C interface: two calls in a row, the second
with a smaller input, bit-exact; the size limit of its static scratch; its error word."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1507_01391_amd import inputs

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 32 << 20


@pytest.fixture(scope="module")
def ts():
    import paper_1507_01391_amd as ts
    return ts


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def noalloc_sort(keys, payload, off, max_len, schedule="auto", err=None):
    """One tile_sort_noalloc call with freshly allocated outputs (allocated here, by
    the caller, before the call)."""
    from paper_1507_01391_amd import _lib
    lib = _lib.load()
    n = keys.shape[0]
    ch, es, cs = (0, 1, 0) if payload is None else ((1, 1, 0) if payload.dim() == 1 else (payload.shape[0], 1, n))
    ko = torch.empty_like(keys)
    po = None if payload is None else torch.empty_like(payload)
    pm = torch.empty(n, dtype=torch.int32, device="cuda")
    _lib.check(lib.tile_sort_noalloc(_p(keys), _p(ko), _p(payload), _p(po), ch, es, cs, _p(pm), _p(off),
                                     off.numel() - 1, n, max_len, _lib.sched_flags(schedule), _p(err),
                                     _stream()))
    return ko, po, pm


def ref_sort(ts, keys, payload, off, max_len, schedule="auto"):
    return ts.tile_sort(keys, payload, off, max_tile_len=max_len, schedule=schedule)


def _same(a, b):
    return a is None and b is None or torch.equal(a, b)


@pytest.mark.parametrize("schedule", ["auto", "merge", "split"])
def test_noalloc_matches_tile_sort_twice(ts, schedule):
    from tests.gpu_util import dev
    cap = 32768 if schedule != "split" else 16384
    # first call: uneven segments with every key distribution and a 2-channel payload
    k1, p1, o1, _ = inputs.segments(seed=71, num_segments=400, hi=cap)
    p1 = np.stack([p1, p1 ^ np.uint32(0x5A5A5A5A)])
    # second call, smaller: fewer, shorter segments and one channel
    k2, p2, o2, _ = inputs.segments(seed=72, num_segments=37, hi=cap // 4)
    for keys, pay, off, ml in ((k1, p1, o1, cap), (k2, p2, o2, cap // 4)):
        d_k, d_p, d_o = dev(keys), dev(pay), dev(off)
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        got = noalloc_sort(d_k, d_p, d_o, ml, schedule, err)
        want = ref_sort(ts, d_k, d_p, d_o, ml, schedule)
        ts.check_device_errors()
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        for g, w in zip(got, want):
            assert _same(g, w)


def test_noalloc_without_perm_payload_uses_scratch_permutation(ts):
    """A payload without perm_out keeps the permutation in the scratch (split schedule
    with a large batch: routed gather)."""
    from paper_1507_01391_amd import _lib
    from tests.gpu_util import dev
    lib = _lib.load()
    rng = np.random.default_rng(73)
    sizes = rng.integers(1, 4097, size=1500)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(off[-1])
    keys = rng.integers(0, 100, size=n, dtype=np.uint32)
    pay = rng.integers(0, 2**32, size=n, dtype=np.uint32)
    d_k, d_p, d_o = dev(keys), dev(pay), dev(off)
    ko, po = torch.empty_like(d_k), torch.empty_like(d_p)
    for _ in range(2):
        _lib.check(lib.tile_sort_noalloc(_p(d_k), _p(ko), _p(d_p), _p(po), 1, 1, 0, None, _p(d_o), len(sizes), n,
                                         4096, _lib.sched_flags("split"), None, _stream()))
        wk, wp, _ = ref_sort(ts, d_k, d_p, d_o, 4096, "split")
        torch.cuda.synchronize()
        assert torch.equal(ko, wk) and torch.equal(po, wp)


def test_noalloc_rejects_calls_beyond_its_scratch(ts):
    """The merge schedule with a tile above 32768 keys keeps 16-byte runs per key: far
    beyond the 32 MiB scratch for 2^22 keys.  Refused on the host, nothing launched."""
    from paper_1507_01391_amd import _lib
    lib = _lib.load()
    n = 1 << 22
    merge = _lib.sched_flags("merge")
    assert lib.ts_workspace_bytes(0, merge, 1, n, n, 0) > SCRATCH_BYTES
    fake = ctypes.c_void_p(0x1000)
    rc = lib.tile_sort_noalloc(fake, ctypes.c_void_p(0x2000), None, None, 0, 1, 0, None, fake, 1, n, n, merge,
                               None, _stream())
    assert rc == _lib.TS_ERR_WORKSPACE
    assert "32 MiB" in lib.ts_last_error().decode() or str(SCRATCH_BYTES) in lib.ts_last_error().decode()


def test_noalloc_reports_contract_violations_in_err_out(ts):
    from tests.gpu_util import dev
    keys = dev(np.arange(8192, dtype=np.uint32)[::-1].copy())
    off = dev(np.array([0, 8192], np.int64))
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    # max_tile_len understates the tile: the kernel skips it and flags it
    noalloc_sort(keys, None, off, 4096, "bitonic", err)
    torch.cuda.synchronize()
    assert int(err.item()) & 1
    # the next call starts from a clear error word in the scratch
    err2 = torch.zeros(1, dtype=torch.int32, device="cuda")
    ko, _, _ = noalloc_sort(keys, None, off, 8192, "bitonic", err2)
    torch.cuda.synchronize()
    assert int(err2.item()) == 0
    assert torch.equal(ko.cpu(), torch.arange(8192, dtype=torch.int32))
