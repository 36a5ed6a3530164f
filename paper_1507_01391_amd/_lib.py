"""ctypes binding of libtilesort.so (argument marshalling only).

The library is loaded from this package directory.  If it is missing the
import of any op fails loudly: there is no CPU fallback on the product path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtilesort.so")

TS_OK, TS_ERR_INVALID, TS_ERR_UNSUPPORTED, TS_ERR_HIP, TS_ERR_WORKSPACE = range(5)
TS_SCATTER, TS_GATHER = 0, 1
TS_FLAG_F32_ORDERED = 1
TS_FLAG_VALIDATE = 2
TS_FLAG_PI_U16 = 4
TS_FLAG_INV_U16 = 8
SCHED = {"auto": 0, "split": 1, "thm2": 2, "bitonic": 3, "merge": 4, "naive": 15}
TS_OP_SORT, TS_OP_PARTITION, TS_OP_PERMUTE, TS_OP_DEVICE_SORT, TS_OP_DEVICE_PARTITION = 0, 1, 2, 3, 4

# Every symbol include/tilesort.h declares.
EXPORTS = (
    "tile_sort", "tile_partition", "tile_permute", "ts_device_sort", "ts_device_partition",
    "ts_workspace_bytes", "ts_workspace_init",
    "ts_check", "ts_last_error", "ts_version", "ts_copy", "ts_lds_probe", "ts_tune",
    "tile_sort_noalloc",
)


class TileSortError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[status {status}] {message}")
        self.status = status


_lib = None


def sched_flags(schedule: str) -> int:
    return SCHED[schedule] << 8


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python -m paper_1507_01391_amd.build` "
            "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, U32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
    S = ctypes.c_int
    lib.tile_sort.argtypes = [P, P, P, P, U32, I64, I64, P, P, I64, I64, I64, U32, P, SZ, P]
    lib.tile_partition.argtypes = [P, P, P, P, U32, I64, I64, U32, P, P, I64, I64, U32, P, SZ, P]
    lib.tile_sort_noalloc.argtypes = [P, P, P, P, U32, I64, I64, P, P, I64, I64, I64, U32, P, P]
    lib.tile_sort_noalloc.restype = S
    lib.tile_permute.argtypes = [P, P, U32, I64, I64, P, P, P, U32, P, P, I64, I64, U32, P, SZ, P]
    lib.ts_device_sort.argtypes = [P, P, P, P, P, I64, U32, P, SZ, P]
    lib.ts_device_partition.argtypes = [P, P, P, P, P, I64, U32, U32, P, SZ, P]
    for f in ("tile_sort", "tile_partition", "tile_permute", "ts_device_sort", "ts_device_partition"):
        getattr(lib, f).restype = S
    lib.ts_workspace_bytes.argtypes = [ctypes.c_int, U32, I64, I64, I64, U32]
    lib.ts_workspace_bytes.restype = SZ
    lib.ts_workspace_init.argtypes = [P, SZ, P]
    lib.ts_workspace_init.restype = S
    lib.ts_check.argtypes = [P, P]
    lib.ts_check.restype = S
    lib.ts_last_error.argtypes = []
    lib.ts_last_error.restype = ctypes.c_char_p
    lib.ts_version.argtypes = []
    lib.ts_version.restype = ctypes.c_char_p
    lib.ts_copy.argtypes = [P, P, SZ, P]
    lib.ts_copy.restype = S
    lib.ts_lds_probe.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, P, P, P]
    lib.ts_lds_probe.restype = S
    lib.ts_tune.argtypes = [ctypes.c_char_p, ctypes.c_int]
    lib.ts_tune.restype = S
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != TS_OK:
        msg = load().ts_last_error().decode(errors="replace")
        raise TileSortError(status, msg)
