"""Fixed workloads for hardware-counter runs (rocprofv3 --pmc / --kernel-trace).

Each subcommand builds one seeded synthetic workload, runs the chosen operation once
untimed and then `--reps` more times, and exits; every dispatch is a sample for the
profiler.  The LDS bank-model probe issues one throughput dispatch per access pattern
in a fixed order, so counter rows map to patterns by dispatch order (PROBE_PATTERNS).

    python -m paper_1507_01391_amd.profile_run partition --schedule split --tiles 16384
    python -m paper_1507_01391_amd.profile_run permute --schedule split --direction gather
    python -m paper_1507_01391_amd.profile_run permute --n 16384 --tiles 1024 --channels 8
    python -m paper_1507_01391_amd.profile_run permute_fwd_bwd --tiles 16384
    python -m paper_1507_01391_amd.profile_run sort_payload --rows 4096
    python -m paper_1507_01391_amd.profile_run sort --schedule bitonic --tiles 16384
    python -m paper_1507_01391_amd.profile_run segments --segments 20000
    python -m paper_1507_01391_amd.profile_run device_sort --n 268435456 --payload
    python -m paper_1507_01391_amd.profile_run copy --bytes 1073741824
    python -m paper_1507_01391_amd.profile_run probe
"""
from __future__ import annotations

import argparse
import sys

import numpy as np
import torch

from . import inputs, ops

_L = list(range(64))

# (name, op, width in words, per-lane 32-bit word addresses) -- probes of the LDS bank
# structure: strides, lanes l and l+32 (or l+16) on one bank, broadcasts, 64/128-bit
# accesses split in halves / quarters / eighths on the same banks, ds_bpermute.
PROBE_PATTERNS = [
    ("r32_lin", "read", 1, [l for l in _L]),
    ("r32_s2", "read", 1, [2 * l for l in _L]),
    ("r32_s4", "read", 1, [4 * l for l in _L]),
    ("r32_s16", "read", 1, [16 * l for l in _L]),
    ("r32_s32", "read", 1, [32 * l for l in _L]),
    ("r32_s64", "read", 1, [64 * l for l in _L]),
    ("r32_l_and_l+32_same_bank64", "read", 1, [64 * (l // 32) + l % 32 for l in _L]),
    ("r32_even_odd", "read", 1, [2 * (l % 32) + l // 32 for l in _L]),
    ("r32_l_and_l+16_same_bank32", "read", 1, [32 * (l // 16 % 2) + (l % 16) + 64 * (l // 32) for l in _L]),
    ("r32_broadcast", "read", 1, [0 for _ in _L]),
    ("r32_half_broadcast", "read", 1, [l % 32 for l in _L]),
    ("r32_pitch65_transpose", "read", 1, [65 * 7 + l for l in _L]),
    ("w32_lin", "write", 1, [l for l in _L]),
    ("w32_s64", "write", 1, [64 * l for l in _L]),
    ("w32_l_and_l+32_same_bank64", "write", 1, [64 * (l // 32) + l % 32 for l in _L]),
    ("w32_even_odd", "write", 1, [2 * (l % 32) + l // 32 for l in _L]),
    ("w32_same_word", "write", 1, [5 for _ in _L]),
    ("w32_pitch65_transpose", "write", 1, [65 * l + 7 for l in _L]),
    ("r64_lin", "read", 2, [2 * l for l in _L]),
    ("r64_halves_same_banks", "read", 2, [2 * (l % 32) + 128 * (l // 32) for l in _L]),
    ("r64_quarters_same_banks", "read", 2, [2 * (l % 16) + 128 * (l // 16) for l in _L]),
    ("r64_eighths_same_banks", "read", 2, [2 * (l % 8) + 128 * (l // 8) for l in _L]),
    ("r64_s64", "read", 2, [128 * l for l in _L]),
    ("w64_lin", "write", 2, [2 * l for l in _L]),
    ("w64_halves_same_banks", "write", 2, [2 * (l % 32) + 128 * (l // 32) for l in _L]),
    ("w64_quarters_same_banks", "write", 2, [2 * (l % 16) + 128 * (l // 16) for l in _L]),
    ("r128_lin", "read", 4, [4 * l for l in _L]),
    ("r128_eighths_same_banks", "read", 4, [4 * (l % 8) + 256 * (l // 8) for l in _L]),
    ("r128_sixteenths_same_banks", "read", 4, [4 * (l % 16) + 256 * (l // 16) for l in _L]),
    ("w128_lin", "write", 4, [4 * l for l in _L]),
    ("bpermute_lin", "bpermute", 1, [l for l in _L]),
    ("bpermute_rand", "bpermute", 1, [(l * 37 + 11) % 64 for l in _L]),
    ("bpermute_same", "bpermute", 1, [3 for _ in _L]),
]


def _dev(a: np.ndarray) -> torch.Tensor:
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _repeat(fn, reps: int) -> None:
    for _ in range(reps + 1):
        fn()
    torch.cuda.synchronize()


def run_partition(a):
    labels, payload, off = inputs.partition(num_tiles=a.tiles, n=a.n)
    dl, dp, do = _dev(labels), _dev(payload), _dev(off)
    lo, po = torch.empty_like(dl), torch.empty_like(dp)
    _repeat(lambda: ops.tile_partition(dl, dp, do, 64, max_tile_len=a.n, schedule=a.schedule,
                                       labels_out=lo, payload_out=po), a.reps)


def run_permute(a):
    x, pi, _, off = inputs.permutation(num_tiles=a.tiles, n=a.n, family=a.family)
    if a.channels > 1:   # channel-planar payload: x, -x, 2x, ...
        x = np.stack([x * (1 + c // 2) * (-1) ** c for c in range(a.channels)]).astype(np.float32)
    dx, dpi, do = _dev(x), _dev(pi), _dev(off)
    y = torch.empty_like(dx)
    _repeat(lambda: ops.tile_permute(dx, dpi, a.direction, do, max_tile_len=a.n, out=y,
                                     schedule=a.schedule), a.reps)


def run_permute_fwd_bwd(a):
    """Forward scatter writing a 16-bit inverse, backward scatter by it: the path of
    autograd.Permute (and of the fwd+bwd permutation workload of bench.py)."""
    x, pi, g, off = inputs.permutation(num_tiles=a.tiles, n=a.n, family=a.family)
    dx, dpi, dg, do = _dev(x), _dev(pi), _dev(g), _dev(off)
    y, gx = torch.empty_like(dx), torch.empty_like(dx)
    inv = torch.empty(dpi.shape, dtype=torch.int16, device=dpi.device)

    def step():
        ops.tile_permute(dx, dpi, "scatter", do, max_tile_len=a.n, out=y, inv_out=inv)
        ops.tile_permute(dg, inv, "scatter", do, max_tile_len=a.n, out=gx)
    _repeat(step, a.reps)


def run_sort_payload(a):
    """Differentiable sort of rows of fp32 keys with an 8-channel planar payload, forward
    and backward (the path of bench.py's sort-with-payload workload)."""
    from .autograd import sort_with_payload
    keys, payload, grad, off = inputs.sort_payload(rows=a.rows, n=a.n)
    dk = _dev(keys).view(torch.float32).requires_grad_(True)
    dp = _dev(payload).view(torch.float32).requires_grad_(True)
    dg, do = _dev(grad).view(torch.float32), _dev(off)
    gk = torch.ones_like(dk)

    def step():
        sk, sp, _ = sort_with_payload(dk, dp, do, a.n)
        torch.autograd.backward([sk, sp], [gk, dg])
        dk.grad = None
        dp.grad = None
    _repeat(step, a.reps)


def run_sort(a):
    rng = np.random.default_rng(inputs.SEED_BASE + 1)
    keys = rng.integers(0, 2**32, size=a.tiles * a.n, dtype=np.uint32)
    payload = np.tile(np.arange(a.n, dtype=np.uint32), a.tiles)
    off = np.arange(a.tiles + 1, dtype=np.int64) * a.n
    dk, dp, do = _dev(keys), _dev(payload), _dev(off)
    ko, po, pm = torch.empty_like(dk), torch.empty_like(dp), torch.empty_like(dk)
    _repeat(lambda: ops.tile_sort(dk, dp if a.payload else None, do, max_tile_len=a.n,
                                  schedule=a.schedule, keys_out=ko,
                                  payload_out=po if a.payload else None, perm_out=pm), a.reps)


def run_segments(a):
    keys, payload, off, _ = inputs.segments(num_segments=a.segments)
    dk, dp, do = _dev(keys), _dev(payload), _dev(off)
    ko, po, pm = torch.empty_like(dk), torch.empty_like(dp), torch.empty_like(dk)
    _repeat(lambda: ops.tile_sort(dk, dp, do, max_tile_len=32768, schedule=a.schedule,
                                  keys_out=ko, payload_out=po, perm_out=pm), a.reps)


def run_device_sort(a):
    rng = np.random.default_rng(inputs.SEED_BASE + 6)
    keys = _dev(rng.integers(0, 2**32, size=a.n, dtype=np.uint32))
    pay = torch.arange(a.n, dtype=torch.int32, device="cuda") if a.payload else None
    ko = torch.empty_like(keys)
    po = torch.empty_like(keys) if a.payload else None
    _repeat(lambda: ops.device_sort(keys, pay, keys_out=ko, payload_out=po), a.reps)


def run_copy(a):
    src = torch.empty(a.bytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    _repeat(lambda: ops.copy(src, dst), a.reps)


def run_probe(a):
    for name, op, width, lw in PROBE_PATTERNS:
        ops.lds_probe(lw, op=op, width=width, iters=256, waves=16, groups=512)
        torch.cuda.synchronize()
        print(name, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    p = sub.add_parser("partition")
    p.add_argument("--schedule", default="split")
    p.add_argument("--tiles", type=int, default=16384)
    p.add_argument("--n", type=int, default=4096)
    p = sub.add_parser("permute")
    p.add_argument("--schedule", default="split")
    p.add_argument("--direction", default="scatter", choices=["scatter", "gather"])
    p.add_argument("--family", default="uniform")
    p.add_argument("--tiles", type=int, default=4096)
    p.add_argument("--n", type=int, default=8192)
    p.add_argument("--channels", type=int, default=1)
    p = sub.add_parser("permute_fwd_bwd")
    p.add_argument("--family", default="uniform")
    p.add_argument("--tiles", type=int, default=16384)
    p.add_argument("--n", type=int, default=8192)
    p = sub.add_parser("sort_payload")
    p.add_argument("--rows", type=int, default=4096)
    p.add_argument("--n", type=int, default=16384)
    p = sub.add_parser("sort")
    p.add_argument("--schedule", default="bitonic")
    p.add_argument("--tiles", type=int, default=16384)
    p.add_argument("--n", type=int, default=4096)
    p.add_argument("--payload", action="store_true")
    p = sub.add_parser("segments")
    p.add_argument("--schedule", default="merge")
    p.add_argument("--segments", type=int, default=20000)
    p = sub.add_parser("device_sort")
    p.add_argument("--n", type=int, default=1 << 28)
    p.add_argument("--payload", action="store_true")
    p = sub.add_parser("copy")
    p.add_argument("--bytes", type=int, default=1 << 30)
    sub.add_parser("probe")
    for sp in sub.choices.values():
        sp.add_argument("--reps", type=int, default=2)
    a = ap.parse_args(argv)
    {"partition": run_partition, "permute": run_permute, "permute_fwd_bwd": run_permute_fwd_bwd,
     "sort_payload": run_sort_payload, "sort": run_sort,
     "segments": run_segments, "device_sort": run_device_sort, "copy": run_copy, "probe": run_probe}[a.cmd](a)
    print(f"done {a.cmd}", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
