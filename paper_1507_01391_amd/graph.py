"""Capture one tile operation's launch sequence into a HIP graph and replay it.

Every entry point of libtilesort.so enqueues a fixed sequence of kernel launches on
the caller's stream, with no host synchronisation, no allocation and no memset node
(work counters are cleared by a fill kernel), so a stream capture records it as is.
Replaying the graph then costs one launch for the whole batch, whatever the number of
tiles and schedules inside.

The captured kernels keep raw pointers to the buffers given at capture time and to
the library workspace of that moment; the graph object holds references to all of
them so they stay allocated while it lives.
"""
from __future__ import annotations

from typing import Callable, Optional

import torch

from . import ops


class TileGraph:
    """Record `fn()` (calls into this package on the current device) once, replay many.

    `fn` is first run eagerly on a side stream (`warmup` times) so that the workspace
    has reached its final size and launch parameters are cached; the capture follows.
    """

    def __init__(self, fn: Callable[[], object], warmup: int = 1, keep: Optional[list] = None):
        self.fn = fn
        dev = torch.cuda.current_device()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(max(1, warmup)):
                self.result = fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.result = fn()
        self._keep = [ops.workspace(dev)] + list(keep or [])

    def replay(self):
        """Enqueue the recorded launches on the current stream; returns fn's result
        tensors (the same objects every time)."""
        self.graph.replay()
        return self.result


def sort_graph(keys: torch.Tensor, offsets: torch.Tensor, max_tile_len: int,
               payload: Optional[torch.Tensor] = None, f32_ordered: bool = False,
               schedule: str = "auto") -> TileGraph:
    """A graph of one tile_sort over fixed buffers: replay() returns
    (keys_out, payload_out, perm) for whatever `keys` / `payload` hold then."""
    keys_out = torch.empty_like(keys)
    perm = torch.empty(keys.shape[0], dtype=torch.int32, device=keys.device)
    payload_out = None if payload is None else torch.empty_like(payload)

    def fn():
        return ops.tile_sort(keys, payload, offsets, max_tile_len=max_tile_len,
                             f32_ordered=f32_ordered, schedule=schedule, keys_out=keys_out,
                             payload_out=payload_out, perm_out=perm)

    return TileGraph(fn, keep=[keys, offsets, payload])
