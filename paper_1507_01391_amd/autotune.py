"""Autotuner for the kernel-selection table of libtilesort.so.

For every knob (see ts_tune in include/tilesort.h) the tuner times each admissible
value on a synthetic batch of the shape the knob governs, keeps the fastest, and
writes the choices to a JSON plan keyed by GPU architecture.  Importing the package
applies the saved plan for the GPU it runs on (``apply_saved_plan``).

Candidates are the bank-conflict-free schedules only; the naive-LDS baseline is
timed for reference (``baseline_ms``) but never chosen.

    python -m paper_1507_01391_amd.autotune [--out PATH] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import time
from typing import Callable, Dict, Optional

import numpy as np
import torch

from . import ops

PLAN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plans")

# knob -> (candidate values, default)
SORT = {"split": 1, "thm2": 2, "bitonic": 3, "merge": 4, "naive": 15}
KNOBS = {
    "sort_plan_4096": ([SORT["bitonic"], SORT["merge"], SORT["split"], SORT["thm2"]], SORT["bitonic"]),
    "sort_plan_8192": ([SORT["merge"], SORT["split"], SORT["bitonic"], SORT["thm2"]], SORT["merge"]),
    "sort_plan_16384": ([SORT["merge"], SORT["split"], SORT["bitonic"], SORT["thm2"]], SORT["merge"]),
    "merge_pack": ([1, 0], 1),
    "merge_wide": ([32768, 16384, 8192, 4096], 32768),
    "oneshot": ([1, 0], 1),
    "partition_waves_4096": ([168, 176, 166, 164, 106, 108, 104], 168),
    "permute_variant": ([6, 7, 8, 9, 10, 11, 12, 13, 1, 0, 2], 6),
}


def arch_name(device: int = 0) -> str:
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def plan_path(arch: str) -> str:
    return os.environ.get("TS_PLAN_CACHE") or os.path.join(PLAN_DIR, f"{arch}.json")


def apply_plan(plan: Dict[str, int]) -> None:
    for knob, value in plan.items():
        if knob in KNOBS:
            ops.tune(knob, int(value))


def apply_saved_plan() -> Optional[str]:
    """Apply the saved plan of the current GPU's architecture, if there is one.
    Returns the file used, or None (no GPU, or no plan for this architecture)."""
    if not torch.cuda.is_available():
        return None
    path = plan_path(arch_name())
    if not os.path.exists(path):
        return None
    with open(path) as f:
        doc = json.load(f)
    apply_plan(doc.get("plan", {}))
    return path


def _time_ms(fn: Callable[[], object], reps: int) -> float:
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _sizes(rng, tiles: int, lo: int, hi: int) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=tiles)


def _offsets(sizes: np.ndarray) -> np.ndarray:
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def _sort_bench(rng, lo: int, hi: int, keys_total: int, schedule_of: Callable[[int], str],
                log_uniform: bool = False, payload: bool = False):
    if log_uniform:   # segment lengths as in the uneven-segment workload
        mean = (hi - lo) / np.log(hi / lo)
        tiles = max(64, int(keys_total // mean))
        sizes = np.exp(rng.uniform(np.log(lo), np.log(hi + 1), size=tiles)).astype(np.int64).clip(lo, hi)
    else:
        tiles = max(64, keys_total // ((lo + hi) // 2))
        sizes = _sizes(rng, tiles, lo, hi)
    off = _offsets(sizes)
    n = int(off[-1])
    keys = torch.from_numpy(rng.integers(0, 2**32, size=n, dtype=np.uint32).view(np.int32)).cuda()
    pay = torch.arange(n, dtype=torch.int32, device="cuda") if payload else None
    d_off = torch.from_numpy(off).cuda()
    ko, pm = torch.empty_like(keys), torch.empty_like(keys)
    po = torch.empty_like(keys) if payload else None

    def run(value: int):
        return lambda: ops.tile_sort(keys, pay, d_off, max_tile_len=hi, schedule=schedule_of(value),
                                     keys_out=ko, payload_out=po, perm_out=pm)
    return run, n


def tune(quick: bool = False, log=print) -> dict:
    rng = np.random.default_rng(1507)
    total = (1 << 22) if quick else (1 << 25)
    reps = 3 if quick else 5
    inv = {v: k for k, v in SORT.items()}
    plan, timings, baseline = {}, {}, {}

    def choose(knob: str, run_for: Callable[[int], Callable[[], object]], n_items: int,
               set_knob: bool):
        cands, _ = KNOBS[knob]
        best, res = None, {}
        for v in cands:
            if set_knob:
                ops.tune(knob, v)
            ms = _time_ms(run_for(v), reps)
            res[str(v)] = ms
            log(f"[autotune] {knob}={v}: {ms:.3f} ms ({n_items / ms / 1e6:.2f} G items/s)")
            if best is None or ms < res[str(best)]:
                best = v
        plan[knob] = best
        timings[knob] = res
        if set_knob:
            ops.tune(knob, best)

    # tile_sort schedule per length class (explicit schedules, so the plan is not used)
    for knob, lo, hi in (("sort_plan_4096", 2049, 4096), ("sort_plan_8192", 4097, 8192),
                         ("sort_plan_16384", 8193, 16384)):
        run, n = _sort_bench(rng, lo, hi, total, lambda v: inv[v])
        choose(knob, run, n, set_knob=False)
        baseline[knob] = _time_ms(run(SORT["naive"]), reps)
        ops.tune(knob, plan[knob])

    # packing of short tiles in the merge schedule: log-uniform lengths with a payload,
    # as in the uneven-segment workload
    run, n = _sort_bench(rng, 256, 4096, total, lambda v: "merge", log_uniform=True, payload=True)
    choose("merge_pack", run, n, set_knob=True)
    # longest tile the merge schedule sorts whole in one workgroup: the full range of
    # the uneven-segment workload
    run, n = _sort_bench(rng, 256, 32768, total, lambda v: "merge", log_uniform=True, payload=True)
    choose("merge_wide", run, n, set_knob=True)

    # launch shape of the kernels without a variant table: a partition of 2048-item
    # tiles plus a permutation of 4096-item tiles
    tiles = total // 2048
    lab2 = rng.permuted(np.tile(np.repeat(np.arange(64, dtype=np.int32), 32), (tiles, 1)), axis=1)
    d_lab2 = torch.from_numpy(lab2.reshape(-1)).cuda()
    d_pay2 = torch.randn(d_lab2.shape[0], device="cuda")
    d_off2 = torch.arange(tiles + 1, device="cuda", dtype=torch.int64) * 2048
    pi4 = np.argsort(rng.random((total // 4096, 4096)), axis=1).astype(np.int32).reshape(-1)
    d_pi4 = torch.from_numpy(pi4).cuda()
    d_off4 = torch.arange(total // 4096 + 1, device="cuda", dtype=torch.int64) * 4096
    lo2, po2, y4 = torch.empty_like(d_lab2), torch.empty_like(d_pay2), torch.empty_like(d_pay2)

    def shaped():
        ops.tile_partition(d_lab2, d_pay2, d_off2, 64, max_tile_len=2048, labels_out=lo2, payload_out=po2)
        ops.tile_permute(d_pay2, d_pi4, "scatter", d_off4, max_tile_len=4096, out=y4)
    choose("oneshot", lambda v: shaped, 2 * total, set_knob=True)
    del d_lab2, d_pay2, d_off2, d_pi4, d_off4, lo2, po2, y4

    # partition: 4096-item tiles, 64 classes with 64 copies each
    tiles = total // 4096
    lab = np.tile(np.repeat(np.arange(64, dtype=np.int32), 64), (tiles, 1))
    lab = rng.permuted(lab, axis=1).reshape(-1)
    d_lab = torch.from_numpy(lab).cuda()
    d_pay = torch.randn(lab.shape[0], device="cuda")
    d_off = torch.arange(tiles + 1, device="cuda", dtype=torch.int64) * 4096
    lo_, po_ = torch.empty_like(d_lab), torch.empty_like(d_pay)
    choose("partition_waves_4096",
           lambda v: (lambda: ops.tile_partition(d_lab, d_pay, d_off, 64, max_tile_len=4096,
                                                 labels_out=lo_, payload_out=po_)),
           lab.shape[0], set_knob=True)
    baseline["partition_waves_4096"] = _time_ms(
        lambda: ops.tile_partition(d_lab, d_pay, d_off, 64, max_tile_len=4096, schedule="naive",
                                   labels_out=lo_, payload_out=po_), reps)

    # permute: 8192-item tiles, uniform random permutations, forward and backward as
    # autograd.Permute runs them (a scatter writing a 16-bit inverse, a scatter by it)
    tiles = total // 8192
    pi = np.argsort(rng.random((tiles, 8192)), axis=1).astype(np.int32).reshape(-1)
    d_pi = torch.from_numpy(pi).cuda()
    d_x = torch.randn(pi.shape[0], device="cuda")
    d_off = torch.arange(tiles + 1, device="cuda", dtype=torch.int64) * 8192
    y, gx = torch.empty_like(d_x), torch.empty_like(d_x)
    inv = torch.empty(pi.shape[0], dtype=torch.int16, device="cuda")

    def fwd_bwd():
        ops.tile_permute(d_x, d_pi, "scatter", d_off, max_tile_len=8192, out=y, inv_out=inv)
        ops.tile_permute(y, inv, "scatter", d_off, max_tile_len=8192, out=gx)
    choose("permute_variant", lambda v: fwd_bwd, 2 * pi.shape[0], set_knob=True)
    baseline["permute_variant"] = _time_ms(
        lambda: ops.tile_permute(d_x, d_pi, "scatter", d_off, max_tile_len=8192, out=y,
                                 schedule="naive"), reps)

    return {"arch": arch_name(), "device": torch.cuda.get_device_name(0),
            "created": time.strftime("%Y-%m-%d %H:%M:%S"), "quick": quick,
            "plan": plan, "timings_ms": timings, "baseline_ms": baseline}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="plan file (default: plans/<arch>.json)")
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()
    doc = tune(quick=args.quick)
    out = args.out or plan_path(doc["arch"])
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    with open(out, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    print(json.dumps(doc["plan"]))


if __name__ == "__main__":
    main()
