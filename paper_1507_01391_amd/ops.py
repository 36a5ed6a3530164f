"""Torch-facing wrappers of the C interface (argument marshalling only).

Tensors must live on the GPU; every 32-bit dtype (int32, uint32, float32) is
accepted for keys / labels / payload words and moved bit-exactly.  Work is
enqueued on the current torch stream.  Every step of the computation runs in
libtilesort.so; nothing here computes on the host.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib

_WORDS = (torch.int32, torch.float32, torch.uint32)
_DWORDS = (torch.float64, torch.int64)  # moved as two 32-bit words per element
_workspaces: dict = {}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def workspace(device=None, nbytes: int = 0) -> torch.Tensor:
    """Per-device workspace (error word, counters and schedule scratch), zeroed on
    creation.  Grows to at least `nbytes`; the error word is carried over."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else
                       torch.device(device).index or 0)
    ws = _workspaces.get(dev)
    lib = _lib.load()
    need = max(int(nbytes), lib.ts_workspace_bytes(0, 0, 0, 0, 0, 0))
    if ws is None or ws.numel() * 4 < need:
        size = (need + 255) // 256 * 256
        new = torch.empty(size // 4, dtype=torch.int32, device=dev)
        _lib.check(lib.ts_workspace_init(_ptr(new), size, _stream(dev)))
        if ws is not None:
            new[:64].copy_(ws[:64])   # 256-byte header: pending error bits
        _workspaces[dev] = ws = new
    return ws


def check_device_errors(device=None) -> None:
    """Synchronise and raise if a kernel recorded a contract violation."""
    ws = workspace(device)
    _lib.check(_lib.load().ts_check(_ptr(ws), _stream(ws.device)))


def _as_words(t: torch.Tensor, name: str, allow_64: bool = False) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype not in _WORDS and not (allow_64 and t.dtype in _DWORDS):
        raise TypeError(f"{name}: 32-bit dtype required, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _payload_layout(payload: Optional[torch.Tensor], n: int):
    """payload: None, [N] (one channel) or [C, N] channel-planar; 64-bit dtypes are moved
    as two 32-bit words per element.  Returns (channels, es, cs) in 32-bit words."""
    if payload is None:
        return 0, 1, 0
    if payload.dtype in _DWORDS:
        if payload.dim() == 1:
            assert payload.shape[0] == n
            return 2, 2, 1                      # [N, 2] words, array of structs
        assert payload.dim() == 2 and payload.shape[1] == n
        # [C, N] of 64-bit: word (g, c, h) at c*2N + 2g + h -> only one channel group per call
        raise ValueError("64-bit payloads must be 1-D")
    if payload.dim() == 1:
        assert payload.shape[0] == n, "payload length must match keys"
        return 1, 1, 0
    assert payload.dim() == 2 and payload.shape[1] == n, "payload must be [N] or [C, N]"
    return payload.shape[0], 1, n


def _offsets(offsets, n: int, device) -> torch.Tensor:
    if offsets is None:
        return torch.tensor([0, n], dtype=torch.int64, device=device)
    if isinstance(offsets, torch.Tensor):
        assert offsets.dtype == torch.int64
        return offsets.to(device)
    return torch.as_tensor(list(offsets), dtype=torch.int64, device=device)


def longest_tile(offsets) -> int:
    """Longest tile of an offsets tensor (int64, T + 1 entries).  Reads one value back
    from the device, i.e. synchronises; pass max_tile_len to the ops to avoid it."""
    if not isinstance(offsets, torch.Tensor):
        offsets = torch.as_tensor(list(offsets), dtype=torch.int64)
    if offsets.numel() < 2:
        return 0
    return int((offsets[1:] - offsets[:-1]).max().item())


def _max_len(off: torch.Tensor, max_tile_len: Optional[int]) -> int:
    if max_tile_len is not None:
        return int(max_tile_len)
    return longest_tile(off)


def tile_partition(labels: torch.Tensor, payload: Optional[torch.Tensor] = None, offsets=None,
                   num_classes: int = 64, max_tile_len: Optional[int] = None,
                   schedule: str = "auto", want_perm: bool = False, validate: bool = False,
                   labels_out: Optional[torch.Tensor] = None,
                   payload_out: Optional[torch.Tensor] = None,
                   perm_out: Optional[torch.Tensor] = None):
    """Stable w-way partition of every tile (see tile_partition in include/tilesort.h).
    Returns (labels_out, payload_out or None, perm or None)."""
    labels = _as_words(labels, "labels")
    n = labels.shape[0]
    dev = labels.device
    off = _offsets(offsets, n, dev)
    ch, es, cs = _payload_layout(payload, n)
    if payload is not None:
        payload = _as_words(payload, "payload")
        if payload_out is None:
            payload_out = torch.empty_like(payload)
    if labels_out is None:
        labels_out = torch.empty_like(labels)
    if want_perm and perm_out is None:
        perm_out = torch.empty(n, dtype=torch.int32, device=dev)
    flags = _lib.sched_flags(schedule) | (_lib.TS_FLAG_VALIDATE if validate else 0)
    lib = _lib.load()
    T = off.numel() - 1
    ml = _max_len(off, max_tile_len)
    ws = workspace(dev, lib.ts_workspace_bytes(_lib.TS_OP_PARTITION, flags, T, n, ml, ch))
    _lib.check(lib.tile_partition(_ptr(labels), _ptr(labels_out), _ptr(payload), _ptr(payload_out),
                                  ch, es, cs, num_classes, _ptr(perm_out), _ptr(off), T, ml, flags,
                                  _ptr(ws), ws.numel() * 4, _stream(dev)))
    return labels_out, payload_out, perm_out


def tile_permute(x: Optional[torch.Tensor], pi: torch.Tensor, direction: str = "scatter",
                 offsets=None, max_tile_len: Optional[int] = None, schedule: str = "auto",
                 validate: bool = False, out: Optional[torch.Tensor] = None,
                 inv_out: Optional[torch.Tensor] = None, aux: Optional[torch.Tensor] = None,
                 aux_out: Optional[torch.Tensor] = None):
    """Apply tile-local permutations: scatter out[pi[i]] = x[i], gather out[i] = x[pi[i]].
    ``x`` is [N] or [C, N] (channel-planar), or None when only ``inv_out`` (receives
    inv_out[pi[i]] = i from the same routing) is wanted.  ``pi`` and ``inv_out`` are
    int32, or int16 holding the 16-bit tile-local indices.  ``aux`` is an optional extra
    [N] 32-bit tensor moved by the same routing (into ``aux_out``).  Returns ``out``, or
    (``out``, ``aux_out``) when ``aux`` is given."""
    assert pi.dtype in (torch.int32, torch.int16) and pi.is_cuda and pi.is_contiguous()
    n = pi.shape[0]
    dev = pi.device
    if x is not None:
        x = _as_words(x, "x", allow_64=True)
        assert x.shape[-1] == n
        if out is None:
            out = torch.empty_like(x)
    if inv_out is not None:
        assert inv_out.dtype in (torch.int32, torch.int16) and inv_out.shape[0] == n and inv_out.is_contiguous()
    if aux is not None:
        aux = _as_words(aux, "aux")
        assert aux.dim() == 1 and aux.shape[0] == n
        if aux_out is None:
            aux_out = torch.empty_like(aux)
    off = _offsets(offsets, n, dev)
    ch, es, cs = _payload_layout(x, n)
    d = {"scatter": _lib.TS_SCATTER, "gather": _lib.TS_GATHER}[direction]
    ws = workspace(dev)
    flags = _lib.sched_flags(schedule) | (_lib.TS_FLAG_VALIDATE if validate else 0)
    if pi.dtype == torch.int16:
        flags |= _lib.TS_FLAG_PI_U16
    if inv_out is not None and inv_out.dtype == torch.int16:
        flags |= _lib.TS_FLAG_INV_U16
    lib = _lib.load()
    _lib.check(lib.tile_permute(_ptr(x), _ptr(out), ch, es, cs, _ptr(aux), _ptr(aux_out), _ptr(pi), d,
                                _ptr(inv_out), _ptr(off), off.numel() - 1, _max_len(off, max_tile_len),
                                flags, _ptr(ws), ws.numel() * 4, _stream(dev)))
    return out if aux is None else (out, aux_out)


def tile_sort(keys: torch.Tensor, payload: Optional[torch.Tensor] = None, offsets=None,
              max_tile_len: Optional[int] = None, f32_ordered: bool = False,
              schedule: str = "auto", want_perm: bool = True,
              keys_out: Optional[torch.Tensor] = None,
              payload_out: Optional[torch.Tensor] = None,
              perm_out: Optional[torch.Tensor] = None):
    """Stable ascending sort of every tile.  Returns (keys_out, payload_out or None, perm)."""
    keys = _as_words(keys, "keys")
    n = keys.shape[0]
    dev = keys.device
    off = _offsets(offsets, n, dev)
    ch, es, cs = _payload_layout(payload, n)
    if payload is not None:
        payload = _as_words(payload, "payload", allow_64=True)
        if payload_out is None:
            payload_out = torch.empty_like(payload)
    if keys_out is None:
        keys_out = torch.empty_like(keys)
    if want_perm and perm_out is None:
        perm_out = torch.empty(n, dtype=torch.int32, device=dev)
    flags = _lib.sched_flags(schedule) | (_lib.TS_FLAG_F32_ORDERED if f32_ordered else 0)
    lib = _lib.load()
    T = off.numel() - 1
    ml = _max_len(off, max_tile_len)
    ws = workspace(dev, lib.ts_workspace_bytes(_lib.TS_OP_SORT, flags, T, n, ml, ch))
    _lib.check(lib.tile_sort(_ptr(keys), _ptr(keys_out), _ptr(payload), _ptr(payload_out), ch, es,
                             cs, _ptr(perm_out), _ptr(off), T, n, ml, flags, _ptr(ws),
                             ws.numel() * 4, _stream(dev)))
    return keys_out, payload_out, perm_out


def device_sort(keys: torch.Tensor, payload: Optional[torch.Tensor] = None, want_perm: bool = False,
                f32_ordered: bool = False, keys_out: Optional[torch.Tensor] = None,
                payload_out: Optional[torch.Tensor] = None, perm_out: Optional[torch.Tensor] = None):
    """Stable ascending sort of one whole array of 32-bit keys (ts_device_sort): an LSD
    radix sort whose passes are conflict-free 64-way tile partitions.  ``payload`` is an
    optional [N] 32-bit tensor moved with the keys; ``want_perm`` returns the source index
    of every output slot (not together with a payload).  Returns (keys_out, payload_out
    or None, perm or None)."""
    keys = _as_words(keys, "keys")
    assert keys.dim() == 1
    n = keys.shape[0]
    dev = keys.device
    if payload is not None:
        payload = _as_words(payload, "payload")
        assert payload.shape == keys.shape, "one payload word per key"
        if payload_out is None:
            payload_out = torch.empty_like(payload)
    if keys_out is None:
        keys_out = torch.empty_like(keys)
    if want_perm and perm_out is None:
        perm_out = torch.empty(n, dtype=torch.int32, device=dev)
    flags = _lib.TS_FLAG_F32_ORDERED if f32_ordered else 0
    lib = _lib.load()
    carry = 1 if (payload is not None or perm_out is not None) else 0
    ws = workspace(dev, lib.ts_workspace_bytes(_lib.TS_OP_DEVICE_SORT, flags, 1, n, n, carry))
    _lib.check(lib.ts_device_sort(_ptr(keys), _ptr(keys_out), _ptr(payload), _ptr(payload_out),
                                  _ptr(perm_out), n, flags, _ptr(ws), ws.numel() * 4, _stream(dev)))
    return keys_out, payload_out, perm_out


def device_partition(labels: torch.Tensor, payload: Optional[torch.Tensor] = None, num_classes: int = 64,
                     want_perm: bool = False, validate: bool = False,
                     labels_out: Optional[torch.Tensor] = None, payload_out: Optional[torch.Tensor] = None,
                     perm_out: Optional[torch.Tensor] = None):
    """Stable num_classes-way partition of one whole array of labels (ts_device_partition):
    one pass of the device-wide sort with the label as the digit.  ``payload`` is an
    optional [N] 32-bit tensor moved with the labels; ``want_perm`` returns the source
    index of every output slot (not together with a payload).  With ``validate`` a label
    >= num_classes is reported by check_device_errors().  Returns (labels_out,
    payload_out or None, perm or None)."""
    labels = _as_words(labels, "labels")
    assert labels.dim() == 1
    n = labels.shape[0]
    dev = labels.device
    if payload is not None:
        payload = _as_words(payload, "payload")
        assert payload.shape == labels.shape, "one payload word per label"
        if payload_out is None:
            payload_out = torch.empty_like(payload)
    if labels_out is None:
        labels_out = torch.empty_like(labels)
    if want_perm and perm_out is None:
        perm_out = torch.empty(n, dtype=torch.int32, device=dev)
    flags = _lib.TS_FLAG_VALIDATE if validate else 0
    lib = _lib.load()
    ws = workspace(dev, lib.ts_workspace_bytes(_lib.TS_OP_DEVICE_PARTITION, flags, 1, n, n, 0))
    _lib.check(lib.ts_device_partition(_ptr(labels), _ptr(labels_out), _ptr(payload), _ptr(payload_out),
                                       _ptr(perm_out), n, num_classes, flags, _ptr(ws), ws.numel() * 4,
                                       _stream(dev)))
    return labels_out, payload_out, perm_out


def copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    """HBM reference copy (16-byte vector loads and stores)."""
    assert src.is_cuda and dst.is_cuda and src.numel() * src.element_size() <= dst.numel() * dst.element_size()
    lib = _lib.load()
    _lib.check(lib.ts_copy(_ptr(src), _ptr(dst), src.numel() * src.element_size(), _stream(src.device)))


def lds_probe(lane_words: Sequence[int], op: str = "read", width: int = 1, iters: int = 256,
              waves: int = 1, groups: int = 1, device=None):
    """Run the LDS access probe; returns (cycles per wave [tensor], sink)."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    lw = torch.as_tensor(list(lane_words), dtype=torch.int32, device=dev)
    assert lw.numel() == 64
    nw = waves * groups
    cycles = torch.zeros(nw, dtype=torch.int64, device=dev)
    sink = torch.zeros(nw * 64, dtype=torch.int32, device=dev)
    opi = {"read": 0, "write": 1, "bpermute": 2}[op]
    lib = _lib.load()
    _lib.check(lib.ts_lds_probe(_ptr(lw), opi, width, iters, waves, groups, _ptr(cycles),
                                _ptr(sink), _stream(dev)))
    return cycles, sink


_knobs: dict = {}


def tune(knob: str, value: int) -> None:
    """Override one entry of the library's kernel-selection table (see ts_tune)."""
    _lib.check(_lib.load().ts_tune(knob.encode(), int(value)))
    _knobs[knob] = int(value)


def knob(name: str, default: Optional[int] = None) -> Optional[int]:
    """The last value set for a knob through tune() in this process (else `default`)."""
    return _knobs.get(name, default)
