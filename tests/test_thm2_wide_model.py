"""CPU model of the Theorem 2 kernel for 64 x m tiles spread over H = m / 64 wavefronts
(m = 128, 256): the LDS word maps of its moves and exchanges are checked for bounds,
bijectivity and bank conflicts under the measured gfx950 model, and the whole data flow
(register row sorts, exchanges between wavefronts, super-row moves, column sorts, the
final move to store order) is replayed on small-integer inputs with ties and padding and
compared with a stable argsort.

Wavefront h holds columns 64h .. 64h+63 of every row: lane L = row L, register c = column
64h + c.  Theorem 2 (Sec. 2) with super-rows of 8 rows; Lemma 1's condition 8 <= sqrt(m)
holds for every m >= 64.
"""
import numpy as np
import pytest

MOVE_WORDS = 64 * 65
LANES = np.arange(64)


XCH = 32   # registers per exchange round


def wide_words(H):
    return max(64 * (64 * H + 1), H * MOVE_WORDS, H * XCH * 64 * 2)


def move_dst(move, M, L, c):
    """(row, column) destination of (row L, column c) for the super-row moves."""
    i = L & 7
    if move == "RM2CM":
        p = i * M + c
        return (L & ~7) + (p & 7), p >> 3
    p = 8 * c + i
    return (L & ~7) + p // M, p % M


def skew(move, M, cd):
    return cd // (M // 8) if move == "RM2CM" else cd & 7


def write_word(move, M, h, L, c):
    if move == "FINAL":
        return L * (M + 1) + 64 * h + c
    Ld, cd = move_dst(move, M, L, 64 * h + c)
    return cd * 64 + ((Ld + skew(move, M, cd)) & 63)


def read_word(move, M, h, L, c):
    k = 64 * h + c
    if move == "FINAL":
        return 64 * k + L + (64 * k) // M
    return k * 64 + ((L + skew(move, M, k)) & 63)


def conflicts_b32(words):
    """Excess cycles of one 32-bit wave instruction: two 32-lane halves over 32 banks,
    distinct words on one bank conflict (the measured gfx950 model)."""
    extra = 0
    for half in (words[:32], words[32:]):
        banks = {}
        for wd in half:
            banks.setdefault(wd % 32, set()).add(wd)
        extra += max(len(s) for s in banks.values()) - 1
    return extra


@pytest.mark.parametrize("H", [2, 4])
@pytest.mark.parametrize("move", ["RM2CM", "CM2RM", "FINAL"])
def test_wide_moves_bijective_in_bounds_conflict_free(H, move):
    M = 64 * H
    written = {}
    for h in range(H):
        for c in range(64):
            ws = [write_word(move, M, h, L, c) for L in range(64)]
            rs = [read_word(move, M, h, L, c) for L in range(64)]
            assert conflicts_b32(ws) == 0, (h, c)
            assert conflicts_b32(rs) == 0, (h, c)
            assert max(ws + rs) < wide_words(H) and min(ws + rs) >= 0
            for L, wd in enumerate(ws):
                assert wd not in written
                written[wd] = (h, L, c)
    # every read meets exactly the item that the move sends there
    for h in range(H):
        for L in range(64):
            for c in range(64):
                hs, Ls, cs = written[read_word(move, M, h, L, c)]
                if move == "FINAL":
                    # rank Ls*M + 64 hs + cs lands in register c of lane L, wavefront h,
                    # as rank 64 (64 h + c) + L
                    assert Ls * M + 64 * hs + cs == 64 * (64 * h + c) + L
                else:
                    assert move_dst(move, M, Ls, 64 * hs + cs) == (L, 64 * h + c)


@pytest.mark.parametrize("H", [2, 4, 8])
def test_wide_exchange_slots(H):
    """Exchange of XCH registers between wavefronts as 64-bit words: slot (XCH h + j) 64 + L;
    64-bit writes are served 16 lanes at a time, reads 32 lanes at a time, over 64 banks."""
    top = 0
    for h in range(H):
        for j in range(XCH):
            slots = [(XCH * h + j) * 64 + L for L in range(64)]
            top = max(top, 2 * max(slots) + 1)
            for ph in range(0, 64, 16):    # writes: 16 slots = 32 consecutive words
                wd = {(2 * s) % 64 for s in slots[ph:ph + 16]}
                assert len(wd) == 16
            for ph in (0, 32):             # reads: 32 slots distinct modulo 32
                assert len({s % 32 for s in slots[ph:ph + 32]}) == 32
    assert top < max(wide_words(H), H * MOVE_WORDS)


# ---- data flow of the whole kernel ---------------------------------------------------

# composites are key << 30 | position, below 2^62; xor with 2^62 - 1 reverses the order
FULL = np.uint64((1 << 62) - 1)
POS_MASK = np.uint64((1 << 30) - 1)


def mask_of(kind):
    if kind == 0:
        on = np.zeros(64, bool)
    elif kind == 1:
        on = (LANES & 1) == 1
    elif kind == 2:
        on = ((LANES >> 3) & 1) == 1
    else:
        on = ((LANES & 1) ^ ((LANES >> 3) & 1)) == 1
    return np.where(on, FULL, np.uint64(0))


def bitonic_merge_regs(v):
    """In-register ascending bitonic merge over the last axis (stages 32 .. 1)."""
    j = 32
    while j >= 1:
        idx = np.arange(64)
        lo = idx[(idx & j) == 0]
        hi = lo ^ j
        a, b = v[..., lo].copy(), v[..., hi].copy()
        v[..., lo] = np.minimum(a, b)
        v[..., hi] = np.maximum(a, b)
        j //= 2
    return v


def row_sort_regs(v):
    return np.sort(v, axis=-1)


def wide_row_sort(V, H):
    """V[h, L, c]: the steps of the kernel's row sort across H wavefronts."""
    for h in range(H):
        m1 = FULL if h & 1 else np.uint64(0)
        V[h] = row_sort_regs(V[h] ^ m1) ^ m1

    def cross(partner_bit, asc_of):
        W = V.copy()
        for h in range(H):
            hp = h ^ partner_bit
            keep_min = (h < hp) == asc_of(h)
            W[h] = np.minimum(V[h], V[hp]) if keep_min else np.maximum(V[h], V[hp])
        V[:] = W

    asc128 = (lambda h: True) if H == 2 else (lambda h: ((h >> 1) & 1) == 0)
    cross(1, asc128)
    for h in range(H):
        m2 = np.uint64(0) if asc128(h) else FULL
        V[h] = bitonic_merge_regs(V[h] ^ m2) ^ m2
    if H == 4:
        cross(2, lambda h: True)
        cross(1, lambda h: True)
        for h in range(H):
            V[h] = bitonic_merge_regs(V[h])
    return V


def cross_move(V, H, move):
    M = 64 * H
    lds = np.zeros(wide_words(H), dtype=np.uint64)
    for h in range(H):
        for c in range(64):
            for L in range(64):
                lds[write_word(move, M, h, L, c)] = V[h, L, c]
    W = np.empty_like(V)
    for h in range(H):
        for c in range(64):
            for L in range(64):
                W[h, L, c] = lds[read_word(move, M, h, L, c)]
    return W


def transpose_in_wave(V):
    # pitch-65 transpose inside each wavefront: (L, c) -> (c, L)
    return np.ascontiguousarray(np.swapaxes(V, 1, 2))


PHASES = [  # (pre mask, post mask, sort, move), the kernel's phase table
    (1, 1, "row", "RM2CM"), (0, 0, "row", "CM2RM"),
    (1, 1, "row", "RM2CM"), (0, 0, "row", "CM2RM"),
    (0, 0, "row", "T"), (0, 0, "col", "T"),
    (3, 1, "row", "RM2CM"), (0, 0, "row", "CM2RM"),
    (1, 1, "row", "RM2CM"), (0, 0, "row", "CM2RM"),
    (0, 2, "row", "T"), (0, 0, "col", "T"),
    (0, 0, "row", "FINAL"),
]


def run_wide_kernel(keys, H):
    n = len(keys)
    M = 64 * H
    assert n <= 64 * M
    V = np.empty((H, 64, 64), dtype=np.uint64)
    for h in range(H):
        for c in range(64):
            i = 64 * (64 * h + c) + LANES
            k = np.where(i < n, keys[np.minimum(i, max(n - 1, 0))] if n else 0, 0xFFFFFFFF)
            V[h, :, c] = (k.astype(np.uint64) << np.uint64(30)) | i.astype(np.uint64)
    for pre, post, sort, move in PHASES:
        V = V ^ mask_of(pre)[None, :, None]
        V = wide_row_sort(V, H) if sort == "row" else row_sort_regs(V)
        V = V ^ mask_of(post)[None, :, None]
        V = transpose_in_wave(V) if move == "T" else cross_move(V, H, move)
    out = np.empty(64 * M, dtype=np.uint64)
    for h in range(H):
        for c in range(64):
            out[64 * (64 * h + c) + LANES] = V[h, :, c]
    return out[:n]


@pytest.mark.parametrize("H,n,seed,hi", [(2, 8192, 1, 2**32), (2, 5000, 2, 7), (4, 16384, 3, 3),
                                         (4, 9999, 4, 2**32), (2, 1, 5, 9), (4, 64, 6, 1)])
def test_wide_kernel_data_flow_sorts(H, n, seed, hi):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, hi, size=n, dtype=np.uint64).astype(np.uint32)
    out = run_wide_kernel(keys, H)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal((out >> np.uint64(30)).astype(np.uint32), keys[order])
    assert np.array_equal((out & POS_MASK).astype(np.int64), order)


def test_wide_kernel_data_flow_01_inputs():
    """0-1 inputs (the 0-1 principle of Lemma 1's proof) at both widths."""
    rng = np.random.default_rng(11)
    for H in (2, 4):
        for _ in range(3):
            keys = (rng.random(64 * 64 * H) < rng.random()).astype(np.uint32)
            out = run_wide_kernel(keys, H)
            assert np.array_equal((out & POS_MASK).astype(np.int64),
                                  np.argsort(keys, kind="stable"))


# ---- exchange buffer of the bitonic network spread over H wavefronts -----------------
# (its data flow is modelled in test_bitonic_flip_model.py)

def test_wide_exchange_slots_fit_the_transpose_arrays():
    """The exchange buffer of H wavefronts (XCH H x 64 slots of 64 bits) fits in the H
    transpose arrays the wide bitonic sort allocates, for H up to 8."""
    for H in (2, 4, 8):
        top = 2 * ((XCH * (H - 1) + XCH - 1) * 64 + 63) + 1
        assert top < H * MOVE_WORDS


# ---- row sorts that skip levels on runs (the phase table's `runs` field) ------------------

RUNS = [0, 1, 0, 1, 0, 0, 0, 1, 0, 1, 0, 2, 0]   # per phase, as in both kernels' tables


def runs_start(runs, H):
    r = 8 * H if runs == 1 else 8
    return 2 if runs == 0 else min(2 * r, 64)


def network_from(v, start):
    """The kernels' register bitonic network from level `start` on (last axis, 64 items):
    level K sorts K-blocks, ascending where bit K of the index is clear (K = 64: all)."""
    idx = np.arange(64)
    K = start
    while K <= 64:
        j = K // 2
        while j >= 1:
            lo = idx[(idx & j) == 0]
            hi = lo | j
            asc = ((lo & K) == 0) if K < 64 else np.ones(lo.shape, bool)
            a, b = v[..., lo].copy(), v[..., hi].copy()
            mn, mx = np.minimum(a, b), np.maximum(a, b)
            v[..., lo] = np.where(asc, mn, mx)
            v[..., hi] = np.where(asc, mx, mn)
            j //= 2
        K *= 2
    return v


def run_kernel_with_skips(keys, H):
    """The Theorem 2 data flow with every register row sort started at the phase's level
    (64 x 64H tile; H = 1 is the one-wavefront kernel, whose rows need no exchange)."""
    n = len(keys)
    M = 64 * H
    V = np.empty((H, 64, 64), dtype=np.uint64)
    for h in range(H):
        for c in range(64):
            i = 64 * (64 * h + c) + LANES
            k = np.where(i < n, keys[np.minimum(i, max(n - 1, 0))] if n else 0, 0xFFFFFFFF)
            V[h, :, c] = (k.astype(np.uint64) << np.uint64(30)) | i.astype(np.uint64)
    for p, (pre, post, sort, move) in enumerate(PHASES):
        V = V ^ mask_of(pre)[None, :, None]
        start = runs_start(RUNS[p], H)
        if sort == "row":
            for h in range(H):
                m1 = FULL if h & 1 else np.uint64(0)
                V[h] = network_from(V[h] ^ m1, start) ^ m1
            if H > 1:
                # the exchanges and in-register merges of wide_row_sort after the own sort
                W = V.copy()
                asc128 = (lambda h: True) if H == 2 else (lambda h: ((h >> 1) & 1) == 0)
                for h in range(H):
                    hp = h ^ 1
                    keep_min = (h < hp) == asc128(h)
                    W[h] = np.minimum(V[h], V[hp]) if keep_min else np.maximum(V[h], V[hp])
                V = W
                for h in range(H):
                    m2 = np.uint64(0) if asc128(h) else FULL
                    V[h] = bitonic_merge_regs(V[h] ^ m2) ^ m2
                if H == 4:
                    for bit in (2, 1):
                        W = V.copy()
                        for h in range(H):
                            hp = h ^ bit
                            W[h] = np.minimum(V[h], V[hp]) if h < hp else np.maximum(V[h], V[hp])
                        V = W
                    for h in range(H):
                        V[h] = bitonic_merge_regs(V[h])
        else:
            V = network_from(V, start)
        V = V ^ mask_of(post)[None, :, None]
        V = transpose_in_wave(V) if move == "T" else cross_move(V, H, move)
    out = np.empty(64 * M, dtype=np.uint64)
    for h in range(H):
        for c in range(64):
            out[64 * (64 * h + c) + LANES] = V[h, :, c]
    return out[:n]


@pytest.mark.parametrize("H", [1, 2, 4])
@pytest.mark.parametrize("seed,hi", [(1, 2**32), (2, 3), (3, 1)])
def test_row_sorts_started_at_the_runs_level_still_sort(H, seed, hi):
    """Phases 1, 3, 7, 9 see every row (each wavefront's part of it) as runs of 8H items in
    alternating directions, phase 11 every column as runs of 8: starting the register
    network at level 2r there still sorts the tile (full tiles, ties, all-equal keys)."""
    rng = np.random.default_rng(seed * 10 + H)
    n = 4096 * H
    keys = rng.integers(0, hi, size=n, dtype=np.uint64).astype(np.uint32)
    out = run_kernel_with_skips(keys, H)
    assert np.array_equal((out & POS_MASK).astype(np.int64), np.argsort(keys, kind="stable"))


def test_row_sorts_started_at_the_runs_level_ragged():
    rng = np.random.default_rng(17)
    for H, n in ((1, 3000), (2, 5000), (4, 9999), (4, 64)):
        keys = rng.integers(0, 7, size=n, dtype=np.uint64).astype(np.uint32)
        out = run_kernel_with_skips(keys, H)
        assert np.array_equal((out & POS_MASK).astype(np.int64), np.argsort(keys, kind="stable"))


def bitonic_blocks(row, size):
    """Every block of `size` items is strictly ascending then descending, or the reverse,
    with the turn in the middle (two sorted runs of size / 2 in opposite directions)."""
    half = size // 2
    for b in range(0, len(row), size):
        x = np.diff(row[b:b + half].astype(object))
        y = np.diff(row[b + half:b + size].astype(object))
        up_x, dn_x = all(t > 0 for t in x), all(t < 0 for t in x)
        up_y, dn_y = all(t > 0 for t in y), all(t < 0 for t in y)
        if not ((up_x and dn_y) or (dn_x and up_y)):
            return False
    return True


@pytest.mark.parametrize("H", [1, 2, 4])
def test_phase_inputs_are_runs_where_the_table_says(H):
    """The property the kernels rely on, checked directly: at every phase whose `runs` is
    set, the register row each wavefront sorts (after the phase's masks) consists of
    blocks of 2r items that are bitonic (r = 8H after the super-row moves, 8 for the
    column sort), so the network may start at level 2r."""
    rng = np.random.default_rng(23 + H)
    n = 4096 * H
    keys = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    V = np.empty((H, 64, 64), dtype=np.uint64)
    for h in range(H):
        for c in range(64):
            i = 64 * (64 * h + c) + LANES
            V[h, :, c] = (keys[i].astype(np.uint64) << np.uint64(30)) | i.astype(np.uint64)
    for p, (pre, post, sort, move) in enumerate(PHASES):
        V = V ^ mask_of(pre)[None, :, None]
        if RUNS[p]:
            size = runs_start(RUNS[p], H)
            for h in range(H):
                m1 = FULL if (sort == "row" and h & 1) else np.uint64(0)
                W = V[h] ^ m1
                assert all(bitonic_blocks(W[L], size) for L in range(64)), (p, h)
        if sort == "row":
            V = wide_row_sort(V, H) if H > 1 else row_sort_regs(V)
        else:
            V = row_sort_regs(V)
        V = V ^ mask_of(post)[None, :, None]
        V = transpose_in_wave(V) if move == "T" else cross_move(V, H, move)
