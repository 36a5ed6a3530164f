"""CPU oracle: numpy-facing wrappers around ``tilesort_oracle.c``.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
``cpu_baseline`` leg of the benchmark may import this module.  It shares no
code with the HIP library and never imports the product package.

Each function is the plain definition of one problem from Afshani &
Sitchinava, "Sorting and Permuting without Bank Conflicts on GPUs", Sec. 1
("Problems of interest"):

* ``tile_sort``      -- sorting: ascending, ties by position (stable);
* ``tile_partition`` -- w-way partition: group by label, ascending label,
                        input order kept inside a label (the abstract defines
                        partitioning as sorting an input with n/w copies of
                        every label);
* ``tile_permute``   -- permutation: SCATTER out[pi[i]] = in[i],
                        GATHER out[i] = in[pi[i]].

Parity pins (see ``tests/test_oracle_pins.py``): equality with numpy /
Python library sorts, brute force over all orderings and permutations of tiny
tiles, closed forms (identity, transpose, bit reversal), invariants and
hand-worked fixtures in ``tests/golden/``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tilesort_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

SCATTER = 0
GATHER = 1
FLAG_F32_ORDERED = 1

_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP over tiles)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", _SRC,
                               "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        U32 = ctypes.c_uint32
        lib.oracle_f32_order.argtypes = [U32]
        lib.oracle_f32_order.restype = U32
        lib.oracle_f32_order_inv.argtypes = [U32]
        lib.oracle_f32_order_inv.restype = U32
        lib.oracle_tile_sort.argtypes = [P, P, P, P, U32, I64, I64, P, P, I64, U32, ctypes.c_int]
        lib.oracle_tile_sort.restype = ctypes.c_int
        lib.oracle_tile_partition.argtypes = [P, P, P, P, U32, I64, I64, U32, P, P, I64, ctypes.c_int]
        lib.oracle_tile_partition.restype = ctypes.c_int
        lib.oracle_tile_permute.argtypes = [P, P, U32, I64, I64, P, U32, P, I64, ctypes.c_int]
        lib.oracle_tile_permute.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _u32(a):
    a = np.asarray(a)
    if a.dtype == np.float32:
        a = a.view(np.uint32)
    return np.ascontiguousarray(a, dtype=np.uint32)


def _offsets(offsets, n_total):
    if offsets is None:
        offsets = [0, n_total]
    return np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))


def f32_order(bits):
    """Order-preserving uint32 image of float32 bit patterns (scalar or array)."""
    lib = _load()
    if np.isscalar(bits):
        return int(lib.oracle_f32_order(int(bits)))
    b = _u32(bits).ravel()
    return np.array([lib.oracle_f32_order(int(x)) for x in b], dtype=np.uint32).reshape(np.shape(bits))


def f32_order_inv(u):
    lib = _load()
    if np.isscalar(u):
        return int(lib.oracle_f32_order_inv(int(u)))
    b = _u32(u).ravel()
    return np.array([lib.oracle_f32_order_inv(int(x)) for x in b], dtype=np.uint32).reshape(np.shape(u))


def _payload_view(payload, n_total):
    """Return (flat uint32 array, channels, elem_stride, chan_stride) for a payload given as
    None, a 1-D [N] array (one channel), or a 2-D [C, N] channel-planar array."""
    if payload is None:
        return None, 0, 1, 0
    p = _u32(payload)
    if p.ndim == 1:
        assert p.shape[0] == n_total
        return p, 1, 1, 0
    assert p.ndim == 2 and p.shape[1] == n_total, "payload must be [N] or [C, N]"
    return np.ascontiguousarray(p).ravel(), p.shape[0], 1, n_total


def _reshape_payload(flat, payload):
    if flat is None:
        return None
    out = flat.reshape(np.asarray(payload).shape)
    if np.asarray(payload).dtype == np.float32:
        out = out.view(np.float32)
    return out


def tile_sort(keys, payload=None, offsets=None, f32_ordered=False, nthreads=1):
    """Stable ascending sort of every tile.  Returns (keys_out, payload_out, perm).

    ``keys`` is uint32 (or float32 with ``f32_ordered``); ``payload`` is None, [N] or
    [C, N] (channel-planar); ``perm`` holds, per output slot, the tile-local source
    index."""
    lib = _load()
    raw = np.asarray(keys)
    k = _u32(raw)
    n = k.shape[0]
    off = _offsets(offsets, n)
    p, ch, es, cs = _payload_view(payload, n)
    k_out = np.zeros_like(k)
    p_out = None if p is None else np.zeros_like(p)
    perm = np.zeros(n, dtype=np.int32)
    flags = FLAG_F32_ORDERED if f32_ordered else 0
    rc = lib.oracle_tile_sort(_ptr(k), _ptr(k_out), _ptr(p), _ptr(p_out), ch, es, cs, _ptr(perm),
                              _ptr(off), off.shape[0] - 1, flags, nthreads)
    if rc != 0:
        raise ValueError(f"oracle_tile_sort failed: {rc}")
    if raw.dtype == np.float32:
        k_out = k_out.view(np.float32)
    return k_out, _reshape_payload(p_out, payload), perm


def tile_partition(labels, payload=None, offsets=None, num_classes=64, nthreads=1):
    """Stable w-way partition of every tile.  Returns (labels_out, payload_out, perm)."""
    lib = _load()
    lab = _u32(labels)
    n = lab.shape[0]
    off = _offsets(offsets, n)
    p, ch, es, cs = _payload_view(payload, n)
    l_out = np.zeros_like(lab)
    p_out = None if p is None else np.zeros_like(p)
    perm = np.zeros(n, dtype=np.int32)
    rc = lib.oracle_tile_partition(_ptr(lab), _ptr(l_out), _ptr(p), _ptr(p_out), ch, es, cs,
                                   num_classes, _ptr(perm), _ptr(off), off.shape[0] - 1, nthreads)
    if rc == -2:
        raise ValueError("label out of range")
    if rc != 0:
        raise ValueError(f"oracle_tile_partition failed: {rc}")
    return l_out, _reshape_payload(p_out, payload), perm


def tile_permute(x, pi, direction=SCATTER, offsets=None, nthreads=1):
    """Apply a tile-local permutation.  ``x`` is [N] or [C, N]; SCATTER: out[pi[i]] = x[i],
    GATHER: out[i] = x[pi[i]]."""
    lib = _load()
    n = np.asarray(x).shape[-1]
    p, ch, es, cs = _payload_view(x, n)
    pi = np.ascontiguousarray(np.asarray(pi, dtype=np.int32))
    assert pi.shape[0] == n
    off = _offsets(offsets, n)
    out = np.zeros_like(p)
    rc = lib.oracle_tile_permute(_ptr(p), _ptr(out), ch, es, cs, _ptr(pi), direction, _ptr(off),
                                 off.shape[0] - 1, nthreads)
    if rc == -2:
        raise ValueError("pi is not a permutation of its tile")
    if rc != 0:
        raise ValueError(f"oracle_tile_permute failed: {rc}")
    return _reshape_payload(out, x)
