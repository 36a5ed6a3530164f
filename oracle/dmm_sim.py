"""Discrete Memory Machine (DMM) simulator.

TEST INFRASTRUCTURE ONLY (see ``oracle/oracle.py``).  Shares no code with the
HIP library.

Two independent jobs:

1. **The paper's oblivious schedules**, executed literally on a w x m matrix
   whose row i is memory bank i (Afshani & Sitchinava, Sec. 1 "Model of
   Computation"; an array element A[k] lives in row k mod w, column k // w).

   * ``lemma1``   -- the "short and wide" base case of Sec. 2 (Lemma 1): two
                    rounds of {rows in alternating order, row-major to
                    column-major, rows ascending, column-major to row-major},
                    then a final ascending row sort; correct when w <= sqrt(m).
   * ``theorem2`` -- Sec. 2, Theorem 2: super-rows of s adjacent rows sorted by
                    Lemma 1, a column sort, super-rows again in alternating
                    directions, a column sort and a final row sort.  With
                    s = sqrt(m) this is the w = m theorem; with s = sqrt(w) and
                    w <= m it is the w <= m generalisation the abstract claims
                    (a reading; see the design notes).

   The result must be the matrix sorted in row-major order.  Because every
   schedule only looks at relative order, the 0-1 argument of the Lemma 1 and
   Theorem 2 proofs says: sorting every 0/1 input proves the schedule.

2. **Bank-conflict accounting** of address streams.  One *step* is one
   wave-wide memory instruction given as (lane, word address) pairs.  The
   Conflict Avoidance Condition (Sec. 1) demands at most one access per bank
   per step.  ``step_conflicts`` counts the excess in two models:

   * ``"dmm"``      -- strict DMM: every access to an already used bank is a
                       conflict, even to the same word;
   * ``"hardware"`` -- lanes are served in phases of ``phase_lanes`` lanes; an
                       access of ``width`` 32-bit words covers ``width``
                       consecutive banks; inside a phase a bank serving k
                       distinct words costs k - 1 extra cycles (reads of the
                       same word are broadcast for free).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

# --------------------------------------------------------------------------------------------
# 1. Schedules
# --------------------------------------------------------------------------------------------


def row_sort(M: np.ndarray, descending_rows=None) -> np.ndarray:
    """Sort every row of M (each row is one bank, sorted by its own processor).
    ``descending_rows`` is a boolean mask of rows to sort in descending order."""
    out = np.sort(M, axis=1, kind="stable")
    if descending_rows is not None:
        out[descending_rows] = out[descending_rows][:, ::-1]
    return out


def rm_to_cm(M: np.ndarray) -> np.ndarray:
    """Read M in row-major order and refill it column by column: the first w items of the
    first row become the first column, the next w the second column, and so on (Lemma 1,
    step 2).  Item at row-major position p lands at row p mod w, column p // w."""
    w, m = M.shape
    return M.reshape(-1).reshape(m, w).T.copy()


def cm_to_rm(M: np.ndarray) -> np.ndarray:
    """Inverse of ``rm_to_cm``: read M in column-major order and refill it row by row (the
    first m/w columns form the first row; Lemma 1, step 4)."""
    w, m = M.shape
    return M.T.reshape(-1).reshape(w, m).copy()


def lemma1(M: np.ndarray, descending: bool = False, repetitions: int = 2,
           alternate: bool = True, even_rows_ascending: bool = True) -> np.ndarray:
    """Lemma 1 schedule on a w x m matrix (w <= sqrt(m) for correctness).

    Each repetition: rows in alternating order, RM->CM, rows ascending, CM->RM.  Then a
    final ascending row sort.  ``descending`` runs the same schedule with the comparator
    reversed, so the result is sorted descending in row-major order.  The keyword
    arguments exist only so tests can show that each ingredient is needed."""
    w, m = M.shape
    X = -M if descending else M.copy()
    alt = np.zeros(w, dtype=bool)
    if alternate:
        alt[(0 if not even_rows_ascending else 1)::2] = True
    for _ in range(repetitions):
        X = row_sort(X, alt)
        X = rm_to_cm(X)
        X = row_sort(X)
        X = cm_to_rm(X)
    X = row_sort(X)
    return -X if descending else X


def column_sort(M: np.ndarray) -> np.ndarray:
    """Sort every column ascending (top to bottom): transpose, sort rows, transpose."""
    return row_sort(M.T.copy()).T.copy()


def theorem2(M: np.ndarray, s: int | None = None) -> np.ndarray:
    """Theorem 2 schedule.  Super-rows are blocks of ``s`` adjacent rows (default
    s = sqrt(m) as in the theorem, w = m)."""
    w, m = M.shape
    if s is None:
        s = int(round(np.sqrt(m)))
    assert w % s == 0 and s * s <= m, "super-rows need s | w and s <= sqrt(m)"
    X = M.copy()
    groups = [slice(g * s, (g + 1) * s) for g in range(w // s)]
    for g in groups:                     # each super-row sorted by Lemma 1
        X[g] = lemma1(X[g])
    X = column_sort(X)                   # columns ascending
    for gi, g in enumerate(groups):      # super-rows in alternating order
        X[g] = lemma1(X[g], descending=(gi % 2 == 1))
    X = column_sort(X)                   # columns ascending
    return row_sort(X)                   # rows ascending


def is_row_major_sorted(M: np.ndarray) -> bool:
    f = M.reshape(-1)
    return bool(np.all(f[:-1] <= f[1:]))


def all_binary_matrices(w: int, m: int):
    for bits in itertools.product((0, 1), repeat=w * m):
        yield np.array(bits, dtype=np.int64).reshape(w, m)


def random_binary_matrices(w: int, m: int, count: int, seed: int):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        density = rng.random()
        yield (rng.random((w, m)) < density).astype(np.int64)


# --------------------------------------------------------------------------------------------
# 2. Bank-conflict accounting
# --------------------------------------------------------------------------------------------


@dataclass(frozen=True)
class BankModel:
    banks: int = 64          # number of 4-byte banks
    phase_lanes: int = 64    # lanes served together
    width: int = 1           # 32-bit words per lane per access (1, 2 or 4)


def step_conflicts(accesses, model: BankModel, mode: str = "hardware", is_read: bool = True) -> int:
    """Excess cycles of one wave-wide instruction.

    ``accesses`` is an iterable of (lane, word_address) where word_address counts 32-bit
    words and each access covers ``model.width`` consecutive words."""
    acc = sorted(accesses)
    total = 0
    for phase_start in range(0, 64, model.phase_lanes):
        phase = [(l, a) for (l, a) in acc if phase_start <= l < phase_start + model.phase_lanes]
        per_bank: dict[int, list[int]] = {}
        for _, a in phase:
            for k in range(model.width):
                per_bank.setdefault((a + k) % model.banks, []).append(a + k)
        worst = 0
        for words in per_bank.values():
            if mode == "dmm":
                load = len(words)
            elif is_read:
                load = len(set(words))
            else:
                load = len(words)
            worst = max(worst, load)
        total += max(worst - 1, 0)
    return total


# --------------------------------------------------------------------------------------------
# 3. Address model of the alternating-direction binary split (design check)
# --------------------------------------------------------------------------------------------


def binary_split_positions(bits: np.ndarray, base: int, size: int):
    """Destination of every item of one split of a segment of ``size`` items (``size`` a
    multiple of 64) processed in columns of 64 consecutive items: items whose bit is 0 fill
    the segment from the front in their order; items whose bit is 1 fill it from the back,
    in reverse order.  Returns (dest, zeros)."""
    bits = np.asarray(bits).astype(np.int64)
    dest = np.empty(size, dtype=np.int64)
    z = 0
    o = 0
    for v in range(size):
        if bits[v] == 0:
            dest[v] = base + z
            z += 1
        else:
            dest[v] = base + size - 1 - o
            o += 1
    return dest, z


def split_virtual_order(base: int, size: int, zeros: int) -> np.ndarray:
    """Physical position of virtual position v after a split: the zero block is read
    forward, then the one block backward, which restores the stable order."""
    v = np.arange(size)
    return np.where(v < zeros, base + v, base + size - 1 - (v - zeros))
