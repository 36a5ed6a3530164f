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
    assert lib.ts_workspace_bytes(1, 10, 4096, 1) >= 4


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
