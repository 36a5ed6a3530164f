"""Bank-conflict predictions of the naive-LDS permutation kernel from the simulator's
hardware bank model, to set beside the SQ_LDS_BANK_CONFLICT counter of the same
workload (profile_run permute --schedule naive).

TEST INFRASTRUCTURE ONLY (see ``oracle/oracle.py``): it uses ``dmm_sim``'s bank model
and the shared seeded input generator, nothing of the HIP library.

The naive kernel moves one 32-bit word per item through LDS: a scatter writes item
i of a tile to word pi[i] and reads the words back in order; a gather writes in order
and reads word pi[i].  One wave instruction covers 64 consecutive items of the tile
(items 64k .. 64k + 63 for column k), so its word addresses are pi of those items.
In the measured gfx950 model (``profiles/lds_bank_model.md``) a 32-bit access is served
in two 32-lane halves over 32 banks and a bank serving j distinct words costs j - 1
extra cycles; the linear half of each pass has no conflicts.

    python -m oracle.sim_predict --direction scatter --family uniform --tiles 4096
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import dmm_sim  # noqa: E402


def batch_conflicts(words: np.ndarray, model: dmm_sim.BankModel, is_read: bool = True) -> np.ndarray:
    """Extra cycles of every step: ``words`` is [steps, 64] word addresses (lane l in
    column l); the same count as ``dmm_sim.step_conflicts`` in "hardware" mode, for many
    steps at once.  Returns [steps]."""
    words = np.asarray(words, dtype=np.int64)
    S = words.shape[0]
    P = 64 // model.phase_lanes
    w = words.reshape(S, P, model.phase_lanes)
    # every access covers `width` consecutive words
    cov = (w[..., None] + np.arange(model.width)).reshape(S * P, -1)
    if is_read:  # the same word read by several lanes is one access
        cov = np.sort(cov, axis=1)
        keep = np.ones_like(cov, dtype=bool)
        keep[:, 1:] = cov[:, 1:] != cov[:, :-1]
    else:
        keep = np.ones_like(cov, dtype=bool)
    rows = np.repeat(np.arange(S * P), cov.shape[1]).reshape(cov.shape)
    idx = (rows * model.banks + cov % model.banks)[keep]
    counts = np.bincount(idx, minlength=S * P * model.banks).reshape(S * P, model.banks)
    extra = np.maximum(counts.max(axis=1) - 1, 0)
    return extra.reshape(S, P).sum(axis=1)


def naive_permute_conflicts(pi: np.ndarray, n: int, direction: str) -> dict:
    """Predicted SQ_INSTS_LDS-equivalent instruction count and extra cycles for one
    naive permutation launch over tiles of exactly n items (n a multiple of 64)."""
    cols = pi.reshape(-1, 64).astype(np.int64)
    model = dmm_sim.BankModel(32, 32, 1)
    random_part = batch_conflicts(cols, model, is_read=(direction == "gather"))
    linear = batch_conflicts(np.arange(64)[None, :], model)[0] * cols.shape[0]
    return {"instructions": 2 * cols.shape[0], "conflict_cycles": int(random_part.sum() + linear)}


def _inputs_module():
    """The shared seeded input generator, loaded from its file (it imports only numpy),
    without importing the package that holds the HIP library's binding."""
    import importlib.util
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1507_01391_amd", "inputs.py")
    spec = importlib.util.spec_from_file_location("tilesort_inputs", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def main(argv=None) -> None:
    inputs = _inputs_module()
    ap = argparse.ArgumentParser()
    ap.add_argument("--direction", default="scatter", choices=["scatter", "gather"])
    ap.add_argument("--family", default="uniform")
    ap.add_argument("--tiles", type=int, default=4096)
    ap.add_argument("--n", type=int, default=8192)
    a = ap.parse_args(argv)
    _, pi, _, _ = inputs.permutation(num_tiles=a.tiles, n=a.n, family=a.family)
    r = naive_permute_conflicts(pi, a.n, a.direction)
    print(f"naive permute {a.direction} {a.family} {a.tiles} x {a.n}: {r['instructions']} LDS instructions, "
          f"{r['conflict_cycles']} predicted conflict cycles "
          f"({r['conflict_cycles'] / r['instructions']:.4f} per instruction)")


if __name__ == "__main__":
    main()
