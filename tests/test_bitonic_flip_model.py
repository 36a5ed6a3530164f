"""CPU model of the bitonic kernels of bitonic.hpp in their mirror form: the sort of one
wavefront (bitonic_sort4096: 64 lanes x 64 registers, transposes with lane reversal
through a 64 x 65-word array) and the sort spread over H wavefronts (bitonic_sort_wide:
a mirror stage across wavefronts through the exchange buffer, then half-cleaners).
Every LDS word map is checked for bounds, bijectivity and bank conflicts under the
measured gfx950 model, and the data flow is replayed on small-integer composites with
ties and compared with a stable argsort.  No GPU code is involved."""
import numpy as np
import pytest

R = 64
MOVE_WORDS = 64 * 65
XCH = 32
LANES = np.arange(64)


def conflicts_b32(words):
    """Excess cycles of one 32-bit wave instruction (two 32-lane halves over 32 banks)."""
    extra = 0
    for half in (words[:32], words[32:]):
        banks = {}
        for wd in half:
            banks.setdefault(int(wd) % 32, set()).add(int(wd))
        extra += max(len(s) for s in banks.values()) - 1
    return extra


def rev_bit(c, KB):
    return (c >> (KB - 1)) & 1


def write_words(KB, to_rows, c):
    """Words lanes 0..63 write register c to in transpose_rev<KB, to_rows>."""
    base = 63 - LANES if (to_rows and rev_bit(c, KB)) else LANES
    return 65 * base + c


def read_words(KB, to_rows, c):
    base = 63 - LANES if ((not to_rows) and rev_bit(c, KB)) else LANES
    return 65 * c + base


def transpose_rev(V, KB, to_rows):
    """V[lane, register] -> the layout after transpose_rev<KB, to_rows>, through LDS words."""
    A = np.full(MOVE_WORDS, -1, dtype=np.int64)
    out = np.empty_like(V)
    for c in range(R):
        A[write_words(KB, to_rows, c)] = V[:, c]
    for c in range(R):
        out[:, c] = A[read_words(KB, to_rows, c)]
    return out


@pytest.mark.parametrize("KB", range(1, 7))
@pytest.mark.parametrize("to_rows", [False, True])
def test_transpose_rev_words(KB, to_rows):
    seen = set()
    for c in range(R):
        w, r = write_words(KB, to_rows, c), read_words(KB, to_rows, c)
        assert w.min() >= 0 and w.max() < MOVE_WORDS and r.min() >= 0 and r.max() < MOVE_WORDS
        assert conflicts_b32(w) == 0 and conflicts_b32(r) == 0
        seen.update(w.tolist())
    assert len(seen) == 64 * 64                      # every lane and register its own word
    reads = {int(x) for c in range(R) for x in read_words(KB, to_rows, c)}
    assert reads == seen                             # the reads take exactly those words


@pytest.mark.parametrize("KB", range(1, 7))
def test_transpose_rev_layout_and_mirror(KB):
    """Row layout (lane = row r, register = column c, item 64 r + c); after the forward
    transpose register r holds row r with column c at lane c, or 63 - c in the upper half
    of every 2^KB-row block, so an item and its mirror in the block share a lane; the
    backward transpose restores the row layout."""
    item = (64 * LANES[:, None] + np.arange(R)[None, :]).astype(np.int64)
    T = transpose_rev(item, KB, False)
    for r in range(R):
        cols = 63 - LANES if rev_bit(r, KB) else LANES
        assert np.array_equal(T[:, r], 64 * r + cols)
        m = r ^ ((1 << KB) - 1)
        B = 64 << KB
        mirror = (T[:, r] // B) * B + (B - 1 - T[:, r] % B)
        assert np.array_equal(T[:, m], mirror)
    assert np.array_equal(transpose_rev(T, KB, True), item)


def net_stage(V, J):
    """Ascending compare-exchange of registers (i, i ^ J), i < i ^ J, in every lane."""
    V = V.copy()
    for i in range(R):
        l = i ^ J
        if l > i:
            a, b = V[:, i].copy(), V[:, l].copy()
            V[:, i], V[:, l] = np.minimum(a, b), np.maximum(a, b)
    return V


def net_stages(V, J):
    while J >= 1:
        V = net_stage(V, J)
        J //= 2
    return V


def row_sort(V):
    return np.sort(V, axis=1)    # the register network's result: each row ascending


def bitonic_sort4096(V):
    """The mirror-form bitonic sort of one wavefront; returns the store-order layout
    (register c of lane L = rank 64 c + L)."""
    V = row_sort(V)
    for KB in range(1, 7):
        V = transpose_rev(V, KB, False)
        V = net_stage(V, (1 << KB) - 1)
        if KB >= 2:
            V = net_stages(V, 1 << (KB - 2))
        V = transpose_rev(V, KB, True)
        V = net_stages(V, 32)       # row_merge
    return V.T.copy()               # the plain transpose to store order


def composites(keys, base=0):
    pos = np.arange(len(keys), dtype=np.int64) + base
    return (keys.astype(np.int64) << 30) | pos


@pytest.mark.parametrize("seed,hi", [(1, 2**32), (2, 3), (3, 1), (4, 1000)])
def test_bitonic_sort4096_mirror_form_sorts(seed, hi):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, hi, size=4096, dtype=np.uint64)
    V = composites(keys).reshape(64, 64)        # any initial placement
    out = bitonic_sort4096(V)
    ranks = out.T.reshape(-1)                   # rank 64 c + L at [c, L]
    assert np.array_equal(ranks & ((1 << 30) - 1), np.argsort(keys, kind="stable"))


def mirror_reg(round_, j):
    return (j if j < 16 else j + 32) if round_ == 0 else j + 16


def test_cross_wave_mirror_slots():
    """Round r, slot j holds register mirror_reg(r, j); the partner's mirror register
    (63 - c) sits at slot 31 - j; each round covers 32 registers closed under c -> 63 - c,
    and the reads (slot 31 - j at lane 63 - L) are 32 consecutive slots per phase."""
    regs = []
    for r in (0, 1):
        rs = [mirror_reg(r, j) for j in range(32)]
        assert set(rs) == {63 - c for c in rs}
        for j in range(32):
            assert mirror_reg(r, 31 - j) == 63 - mirror_reg(r, j)
        regs += rs
    assert sorted(regs) == list(range(64))
    for h in range(8):
        for j in range(32):
            rd = [(32 * h + 31 - j) * 64 + (63 - L) for L in range(64)]
            for ph in (0, 32):
                assert len({s % 32 for s in rd[ph:ph + 32]}) == 32
            wr = [(32 * h + j) * 64 + L for L in range(64)]
            for ph in range(0, 64, 16):
                assert len({(2 * s) % 64 for s in wr[ph:ph + 16]}) == 16


def cross_wave_mirror(W, h, hp):
    """W[h][L, c] (store order, item 64 c + L) after the mirror stage of h against hp,
    exchanged slot by slot as the kernel does."""
    out = W[h].copy()
    keep_min = h < hp
    for r in (0, 1):
        X = {}
        for wave in (h, hp):
            for j in range(32):
                X[(wave, j)] = W[wave][:, mirror_reg(r, j)].copy()   # slot j, lane L
        for j in range(32):
            c = mirror_reg(r, j)
            y = X[(hp, 31 - j)][63 - LANES]
            out[:, c] = np.minimum(out[:, c], y) if keep_min else np.maximum(out[:, c], y)
    return out


def merge4096(w):
    """bitonic_merge4096 on store order (item 64 c + L): half-cleaners 2048 .. 1."""
    flat = w.T.reshape(-1).copy()
    j = 2048
    idx = np.arange(4096)
    while j >= 1:
        lo = idx[(idx & j) == 0]
        hi = lo | j
        a, b = flat[lo].copy(), flat[hi].copy()
        flat[lo], flat[hi] = np.minimum(a, b), np.maximum(a, b)
        j //= 2
    return flat.reshape(64, 64).T.copy()


def bitonic_sort_wide(keys, H):
    cap = 4096 * H
    k = np.full(cap, 0xFFFFFFFF, dtype=np.uint64)
    k[:len(keys)] = keys
    C = composites(k)
    W = [bitonic_sort4096(C[4096 * h:4096 * (h + 1)].reshape(64, 64)) for h in range(H)]
    kk = 1
    while (1 << kk) <= H:
        W = [cross_wave_mirror(W, h, h ^ ((1 << kk) - 1)) for h in range(H)]
        for b in range(kk - 2, -1, -1):
            W = [np.minimum(W[h], W[h ^ (1 << b)]) if h < (h ^ (1 << b)) else np.maximum(W[h], W[h ^ (1 << b)])
                 for h in range(H)]
        W = [merge4096(w) for w in W]
        kk += 1
    return np.concatenate([w.T.reshape(-1) for w in W])[:len(keys)]


@pytest.mark.parametrize("H,n,hi", [(2, 8192, 2**32), (2, 4097, 5), (4, 16384, 3), (4, 9000, 2**32),
                                    (8, 32768, 2**32), (8, 16385, 17)])
def test_bitonic_sort_wide_mirror_form_sorts(H, n, hi):
    rng = np.random.default_rng(H * 1000 + n)
    keys = rng.integers(0, hi, size=n, dtype=np.uint64)
    out = bitonic_sort_wide(keys, H)
    assert np.array_equal(out & ((1 << 30) - 1), np.argsort(keys, kind="stable"))
