"""MI355X (gfx950) tile sort / w-way partition / permute without LDS bank conflicts.

Afshani & Sitchinava, "Sorting and Permuting without Bank Conflicts on GPUs".
The computation lives in the HIP library ``libtilesort.so`` (C interface in
``include/tilesort.h``); this package is its Python binding.
"""
from .autograd import Permute, SortWithPayload, permute, sort_with_payload
from .ops import (check_device_errors, copy, device_partition, device_sort, knob, lds_probe,
                  tile_partition, tile_permute, tile_sort, tune, workspace)
from .graph import TileGraph, sort_graph
from . import autotune as _autotune

# the autotuned kernel-selection plan of this GPU's architecture, when one is saved
plan_file = _autotune.apply_saved_plan()

__all__ = ["tile_sort", "tile_partition", "tile_permute", "device_sort", "device_partition", "copy",
           "lds_probe", "workspace", "check_device_errors", "tune", "knob", "Permute", "SortWithPayload", "permute",
           "sort_with_payload", "TileGraph", "sort_graph", "plan_file"]
