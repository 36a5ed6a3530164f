"""CPU checks of the C interface: the library loads and exports every declared symbol,
and host-side argument validation rejects bad calls without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "tilesort.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:ts_status|size_t|const char\*)\s+(\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1507_01391_amd import _lib
    return _lib.load()


def test_header_declares_the_three_ops():
    names = declared_functions()
    for f in ("tile_sort", "tile_partition", "tile_permute"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1507_01391_amd import _lib
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTS)
    for f in names:
        assert hasattr(lib, f), f


def test_version_and_workspace_size(lib):
    assert b"gfx950" in lib.ts_version()
    assert lib.ts_workspace_bytes(1, 0, 10, 40960, 4096, 1) >= 256
    # the merge schedule keeps two runs of 8-byte composites plus work lists
    merge = 4 << 8
    n, tiles = 1 << 20, 64
    assert lib.ts_workspace_bytes(0, merge, tiles, n, 65536, 1) >= 16 * n
    # AUTO takes the merge schedule beyond 16384 keys per tile
    assert lib.ts_workspace_bytes(0, 0, tiles, n, 32768, 0) == lib.ts_workspace_bytes(0, merge, tiles, n, 32768, 0)
    assert lib.ts_workspace_bytes(0, 0, tiles, n, 65536, 0) == lib.ts_workspace_bytes(0, merge, tiles, n, 65536, 0)
    # a single piece per tile needs no runs, and neither do tiles sorted whole by one
    # workgroup (up to 32768 keys)
    assert lib.ts_workspace_bytes(0, merge, tiles, n, 4096, 0) < 2 * n
    assert lib.ts_workspace_bytes(0, merge, tiles, n, 32768, 0) < 2 * n
    assert lib.ts_workspace_bytes(0, merge, tiles, n, 32769, 0) >= 16 * n


def _err(lib):
    return lib.ts_last_error().decode()


def test_partition_argument_validation(lib):
    P = ctypes.c_void_p
    fake = P(0x1000)
    ws = P(0x2000)
    # num_classes out of range
    rc = lib.tile_partition(fake, P(0x3000), None, None, 0, 1, 0, 65, None, fake, 1, 4096, 0, ws, 256, None)
    assert rc == 1 and "num_classes" in _err(lib)
    # aliasing
    rc = lib.tile_partition(fake, fake, None, None, 0, 1, 0, 64, None, fake, 1, 4096, 0, ws, 256, None)
    assert rc == 1 and "alias" in _err(lib)
    # missing workspace
    rc = lib.tile_partition(fake, P(0x3000), None, None, 0, 1, 0, 64, None, fake, 1, 4096, 0, None, 0, None)
    assert rc == 4
    # negative tile count
    rc = lib.tile_partition(fake, P(0x3000), None, None, 0, 1, 0, 64, None, fake, -1, 4096, 0, ws, 256, None)
    assert rc == 1
    # tile too long for any kernel
    rc = lib.tile_partition(fake, P(0x3000), None, None, 0, 1, 0, 64, None, fake, 1, 1 << 20, 0, ws, 256, None)
    assert rc == 2
    # Theorem 2 and the bitonic network partition tiles of up to 16384 labels
    thm2, bitonic, naive = 2 << 8, 3 << 8, 15 << 8
    rc = lib.tile_partition(fake, P(0x3000), None, None, 0, 1, 0, 64, None, fake, 1, 16385, thm2, ws, 256, None)
    assert rc == 2
    rc = lib.tile_partition(fake, P(0x3000), None, None, 0, 1, 0, 64, None, fake, 1, 16385, bitonic, ws, 256, None)
    assert rc == 2
    # the naive baseline moves one payload channel; the other schedules any number
    rc = lib.tile_partition(fake, P(0x3000), fake, P(0x4000), 2, 1, 4096, 64, None, fake, 1, 4096, naive, ws,
                            256, None)
    assert rc == 2 and "channel" in _err(lib)
    # partition needs no workspace beyond the error word, whatever the schedule and payload
    for sched in (0, 1 << 8, thm2, bitonic):
        assert lib.ts_workspace_bytes(1, sched, 1000, 1000 * 16384, 16384, 3) == 256


def test_sort_argument_validation(lib):
    P = ctypes.c_void_p
    fake = P(0x1000)
    ws = P(0x2000)
    merge = 4 << 8
    # total_len < 0
    rc = lib.tile_sort(fake, P(0x3000), None, None, 0, 1, 0, None, fake, 1, -1, 4096, 0, ws, 256, None)
    assert rc == 1 and "total_len" in _err(lib)
    # aliasing
    rc = lib.tile_sort(fake, fake, None, None, 0, 1, 0, None, fake, 1, 4096, 4096, 0, ws, 256, None)
    assert rc == 1 and "alias" in _err(lib)
    # the bitonic and Theorem 2 schedules hold 16384 keys per tile
    rc = lib.tile_sort(fake, P(0x3000), None, None, 0, 1, 0, None, fake, 1, 16385, 16385, 3 << 8, ws, 256, None)
    assert rc == 2
    rc = lib.tile_sort(fake, P(0x3000), None, None, 0, 1, 0, None, fake, 1, 16385, 16385, 2 << 8, ws, 256, None)
    assert rc == 2
    # the merge schedule holds 2^28 keys per tile
    rc = lib.tile_sort(fake, P(0x3000), None, None, 0, 1, 0, None, fake, 1, 1 << 29, (1 << 28) + 1, merge,
                       ws, 1 << 40, None)
    assert rc == 2
    # the merge schedule needs its workspace
    rc = lib.tile_sort(fake, P(0x3000), None, None, 0, 1, 0, None, fake, 1, 65536, 65536, merge, ws, 256, None)
    assert rc == 4 and "workspace" in _err(lib)
    # no tiles: nothing to do, nothing launched
    rc = lib.tile_sort(fake, P(0x3000), None, None, 0, 1, 0, None, fake, 0, 0, 0, merge, ws, 256, None)
    assert rc == 0


def test_tune_knob_validation(lib):
    assert lib.ts_tune(b"sort_plan_8192", 3) == 0          # bitonic and Theorem 2 hold 16384 keys
    assert lib.ts_tune(b"sort_plan_16384", 2) == 0
    assert lib.ts_tune(b"sort_plan_16384", 4) == 0
    assert lib.ts_tune(b"sort_plan_8192", 4) == 0
    assert lib.ts_tune(b"sort_plan_8192", 5) == 1          # no such schedule
    assert lib.ts_tune(b"merge_wide", 12288) == 1
    assert lib.ts_tune(b"merge_wide", 32768) == 0
    assert lib.ts_tune(b"sort_plan_4096", 7) == 1
    assert lib.ts_tune(b"merge_pack", 2) == 1
    assert lib.ts_tune(b"no_such_knob", 0) == 1
    assert lib.ts_tune(b"sort_plan_16384", 1) == 0
    assert lib.ts_tune(b"sort_plan_16384", 4) == 0         # back to the default
    assert lib.ts_tune(b"merge_pack", 1) == 0
    for knob, bad, good in ((b"oneshot", 2, 1), (b"naive_oneshot", -1, 0), (b"sort_small_batch", -1, 1024),
                            (b"permute_variant", 14, 6), (b"partition_waves_4096", 110, 168)):
        assert lib.ts_tune(knob, bad) == 1, knob
        assert lib.ts_tune(knob, good) == 0, knob


def test_permute_argument_validation(lib):
    P = ctypes.c_void_p
    fake, ws, pi = P(0x1000), P(0x2000), P(0x4000)
    # inverse output aliasing pi
    rc = lib.tile_permute(fake, P(0x3000), 1, 1, 0, None, None, pi, 0, pi, fake, 1, 4096, 0, ws, 256, None)
    assert rc == 1 and "inv_out" in _err(lib)
    # bad direction
    rc = lib.tile_permute(fake, P(0x3000), 1, 1, 0, None, None, pi, 5, None, fake, 1, 4096, 0, ws, 256, None)
    assert rc == 1 and "direction" in _err(lib)
    # no payload and no inverse wanted: nothing to do
    rc = lib.tile_permute(None, None, 0, 1, 0, None, None, pi, 0, None, fake, 1, 4096, 0, ws, 256, None)
    assert rc == 0
    # tiles longer than the routing capacity
    rc = lib.tile_permute(fake, P(0x3000), 1, 1, 0, None, None, pi, 0, None, fake, 1, 32768, 0, ws, 256, None)
    assert rc == 2
    # the aux channel: both pointers or neither, not aliased, not with the naive schedule
    rc = lib.tile_permute(fake, P(0x3000), 1, 1, 0, P(0x5000), None, pi, 0, None, fake, 1, 4096, 0, ws, 256, None)
    assert rc == 1 and "aux" in _err(lib)
    rc = lib.tile_permute(fake, P(0x3000), 1, 1, 0, P(0x5000), P(0x5000), pi, 0, None, fake, 1, 4096, 0, ws, 256,
                          None)
    assert rc == 1 and "alias" in _err(lib)
    rc = lib.tile_permute(fake, P(0x3000), 1, 1, 0, P(0x5000), P(0x6000), pi, 0, None, fake, 1, 4096, 15 << 8, ws,
                          256, None)
    assert rc == 2 and "aux" in _err(lib)


def test_device_sort_argument_validation(lib):
    P = ctypes.c_void_p
    keys, out, pay, pout, perm, ws = P(0x1000), P(0x2000), P(0x3000), P(0x4000), P(0x5000), P(0x8000)
    big = 1 << 40
    assert lib.ts_device_sort(keys, out, None, None, None, -1, 0, ws, big, None) == 1
    assert lib.ts_device_sort(keys, out, None, None, None, 1 << 31, 0, ws, big, None) == 2
    assert lib.ts_device_sort(keys, keys, None, None, None, 100, 0, ws, big, None) == 1      # alias
    assert lib.ts_device_sort(None, out, None, None, None, 100, 0, ws, big, None) == 1
    assert lib.ts_device_sort(keys, out, pay, None, None, 100, 0, ws, big, None) == 1        # half a payload
    assert lib.ts_device_sort(keys, out, pay, pay, None, 100, 0, ws, big, None) == 1         # payload alias
    assert lib.ts_device_sort(keys, out, pay, pout, perm, 100, 0, ws, big, None) == 2        # payload + perm
    need = lib.ts_workspace_bytes(3, 0, 1, 100, 100, 1)
    assert need >= 256 + 100 * 8
    assert lib.ts_device_sort(keys, out, None, None, perm, 100, 0, ws, need - 1, None) == 4  # workspace
    assert lib.ts_device_sort(keys, out, None, None, None, 0, 0, ws, 0, None) == 0           # empty: nothing to do
    assert lib.ts_device_sort(keys, out, None, None, None, 100, 0, None, big, None) == 4


def test_device_partition_argument_validation(lib):
    P = ctypes.c_void_p
    lab, out, pay, pout, perm, ws = P(0x1000), P(0x2000), P(0x3000), P(0x4000), P(0x5000), P(0x8000)
    big = 1 << 40
    f = lib.ts_device_partition
    assert f(lab, out, None, None, None, -1, 64, 0, ws, big, None) == 1
    assert f(lab, out, None, None, None, 1 << 31, 64, 0, ws, big, None) == 2
    assert f(lab, out, None, None, None, 100, 0, 0, ws, big, None) == 1           # no classes
    assert f(lab, out, None, None, None, 100, 65, 0, ws, big, None) == 1          # more than w
    assert f(lab, lab, None, None, None, 100, 64, 0, ws, big, None) == 1          # alias
    assert f(None, out, None, None, None, 100, 64, 0, ws, big, None) == 1
    assert f(lab, out, pay, None, None, 100, 64, 0, ws, big, None) == 1           # half a payload
    assert f(lab, out, pay, pay, None, 100, 64, 0, ws, big, None) == 1            # payload alias
    assert f(lab, out, pay, pout, perm, 100, 64, 0, ws, big, None) == 2           # payload + perm
    need = lib.ts_workspace_bytes(4, 0, 1, 100, 100, 0)
    assert 256 <= need < lib.ts_workspace_bytes(3, 0, 1, 100, 100, 0)              # no second data copy
    assert f(lab, out, None, None, perm, 100, 64, 0, ws, need - 1, None) == 4     # workspace
    assert f(lab, out, None, None, None, 0, 64, 0, ws, 0, None) == 0              # empty
    assert f(lab, out, None, None, None, 100, 64, 0, None, big, None) == 4
