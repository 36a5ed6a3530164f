"""Pins of the DMM simulator: the paper's schedules under the 0-1 argument of the
Lemma 1 / Theorem 2 proofs, the layout conversions against hand-worked
fixtures, and the bank-conflict accounting on textbook access patterns."""
import json
import os

import numpy as np
import pytest

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_worked.json")))


def test_conversions_golden(sim):
    g = GOLDEN["rm_to_cm_2x4"]
    assert sim.rm_to_cm(np.array(g["M"])).tolist() == g["CM"]
    g = GOLDEN["cm_to_rm_2x4"]
    assert sim.cm_to_rm(np.array(g["M"])).tolist() == g["RM"]


def test_conversion_index_maps(sim):
    """RM->CM sends row-major position p to (p mod w, p // w); CM->RM is its inverse."""
    w, m = 8, 64
    M = np.arange(w * m).reshape(w, m)
    C = sim.rm_to_cm(M)
    for p in range(w * m):
        assert C[p % w, p // w] == p
    assert np.array_equal(sim.cm_to_rm(C), M)


@pytest.mark.parametrize("w,m", [(2, 4), (2, 8)])
def test_lemma1_exhaustive_01(sim, w, m):
    for M in sim.all_binary_matrices(w, m):
        assert sim.is_row_major_sorted(sim.lemma1(M))


@pytest.mark.parametrize("w,m,count", [(4, 16, 3000), (8, 64, 400)])
def test_lemma1_random_01(sim, w, m, count):
    for M in sim.random_binary_matrices(w, m, count, seed=w * m):
        assert sim.is_row_major_sorted(sim.lemma1(M))


def test_lemma1_descending(sim):
    rng = np.random.default_rng(0)
    M = rng.integers(0, 1000, size=(4, 16))
    out = sim.lemma1(M, descending=True).reshape(-1)
    assert np.array_equal(out, np.sort(M.reshape(-1))[::-1])


def test_lemma1_parity_of_alternation_irrelevant(sim):
    for M in sim.all_binary_matrices(2, 8):
        assert sim.is_row_major_sorted(sim.lemma1(M, even_rows_ascending=False))


def test_lemma1_needs_alternation(sim):
    fails = sum(not sim.is_row_major_sorted(sim.lemma1(M, alternate=False))
                for M in sim.all_binary_matrices(2, 8))
    assert fails > 0


def test_lemma1_needs_two_repetitions(sim):
    fails = sum(not sim.is_row_major_sorted(sim.lemma1(M, repetitions=1))
                for M in sim.random_binary_matrices(4, 16, 3000, seed=1))
    assert fails > 0


def test_lemma1_needs_w_le_sqrt_m(sim):
    fails = sum(not sim.is_row_major_sorted(sim.lemma1(M))
                for M in sim.random_binary_matrices(16, 16, 300, seed=2))
    assert fails > 0


@pytest.mark.slow
def test_theorem2_exhaustive_01_4x4(sim):
    for M in sim.all_binary_matrices(4, 4):
        assert sim.is_row_major_sorted(sim.theorem2(M, s=2))


@pytest.mark.parametrize("w,m,s,count", [(16, 16, 4, 400), (64, 64, 8, 60),
                                         (64, 128, 8, 30), (64, 256, 8, 15), (16, 32, 4, 400)])
def test_theorem2_random_01(sim, w, m, s, count):
    for M in sim.random_binary_matrices(w, m, count, seed=w + m + s):
        assert sim.is_row_major_sorted(sim.theorem2(M, s=s))


def test_theorem2_sorts_integers_like_numpy(sim):
    rng = np.random.default_rng(4)
    M = rng.integers(0, 2**32, size=(64, 64), dtype=np.int64)
    assert np.array_equal(sim.theorem2(M).reshape(-1), np.sort(M.reshape(-1)))
    L = rng.integers(0, 64, size=(64, 128))
    assert np.array_equal(sim.theorem2(L, s=8).reshape(-1), np.sort(L.reshape(-1)))


# -------------------------------------------------------------------------- conflict counter


def test_conflicts_linear_and_strided(sim):
    m64 = sim.BankModel(banks=64, phase_lanes=64, width=1)
    lin = [(l, l) for l in range(64)]
    assert sim.step_conflicts(lin, m64) == 0
    strided = [(l, 64 * l) for l in range(64)]
    assert sim.step_conflicts(strided, m64) == 63
    # strided access A[w*i + t] of the Dotsenko layout: lane t only ever touches bank t
    for i in range(5):
        assert sim.step_conflicts([(t, 64 * i + t) for t in range(64)], m64) == 0


def test_conflicts_broadcast_modes(sim):
    m = sim.BankModel(64, 64, 1)
    same = [(l, 17) for l in range(64)]
    assert sim.step_conflicts(same, m, mode="hardware", is_read=True) == 0
    assert sim.step_conflicts(same, m, mode="dmm") == 63


def test_conflicts_padding_coprime(sim):
    """Contiguous access with row length coprime to the bank count is conflict-free."""
    m = sim.BankModel(64, 64, 1)
    for L in (63, 65, 129):
        assert sim.step_conflicts([(t, t * L + 3) for t in range(64)], m) == 0
    assert sim.step_conflicts([(t, t * 64 + 3) for t in range(64)], m) == 63


# ------------------------------------------------------ alternating-direction split (design)


MODELS = [sim_model for sim_model in [
    (64, 64, 1), (32, 32, 1), (64, 32, 2), (32, 16, 2), (64, 16, 4)]]


@pytest.mark.parametrize("banks,phase,width", MODELS)
def test_binary_split_writes_conflict_free(sim, banks, phase, width):
    """Zeros fill a segment from the front, ones from the back: every 64-item column's
    64 destinations are 64 cyclically consecutive slots, hence conflict-free."""
    model = sim.BankModel(banks, phase, width)
    rng = np.random.default_rng(banks + phase + width)
    for trial in range(40):
        size = 64 * int(rng.integers(1, 9))
        base = 64 * int(rng.integers(0, 4))
        bits = (rng.random(size) < rng.random()).astype(int)
        dest, _ = sim.binary_split_positions(bits, base, size)
        for k in range(size // 64):
            acc = [(l, width * int(dest[64 * k + l])) for l in range(64)]
            assert sim.step_conflicts(acc, model, is_read=False) == 0


@pytest.mark.parametrize("banks,phase,width", MODELS)
def test_binary_split_virtual_reads_conflict_free(sim, banks, phase, width):
    model = sim.BankModel(banks, phase, width)
    rng = np.random.default_rng(7)
    for trial in range(40):
        size = 64 * int(rng.integers(1, 9))
        zeros = int(rng.integers(0, size + 1))
        phys = sim.split_virtual_order(0, size, zeros)
        for k in range(size // 64):
            acc = [(l, width * int(phys[64 * k + l])) for l in range(64)]
            assert sim.step_conflicts(acc, model, is_read=True) == 0


def test_binary_split_lsd_is_a_stable_partition(sim):
    """Repeated splits on label bits 0..5, each reading the previous result in its virtual
    order, give the stable partition (compared with numpy's stable argsort)."""
    rng = np.random.default_rng(8)
    n = 4096
    labels = rng.integers(0, 64, size=n)
    order = np.arange(n)              # virtual order -> item id
    for b in range(6):
        bits = (labels[order] >> b) & 1
        dest, zeros = sim.binary_split_positions(bits, 0, n)
        phys = np.empty(n, dtype=np.int64)
        phys[dest] = order            # physical array after the split
        order = phys[sim.split_virtual_order(0, n, zeros)]
    assert np.array_equal(order, np.argsort(labels, kind="stable"))


# ---- layout moves of the register sort (32-bit planes, measured gfx950 model) --------
# 32-bit accesses: two 32-lane halves over 32 banks; the stricter 64-bank / 64-lane DMM
# reading is checked too.
B32_MODELS = [(32, 32), (64, 64)]


def move_dst(move, L, c):
    """Destination (lane, register) of register c of lane L for the three moves."""
    if move == "T":
        return c, L
    if move == "RM2CM":       # 8-row super-row, row-major p = 64 i + c -> column-major
        return (L & ~7) + (c & 7), 8 * (L & 7) + (c >> 3)
    return (L & ~7) + (c >> 3), 8 * (c & 7) + (L & 7)   # CM2RM


def move_skew(move, cd):
    return cd if move == "T" else (cd >> 3 if move == "RM2CM" else cd & 7)


def move_write_word(move, L, c):
    Ld, cd = move_dst(move, L, c)
    if move == "T":
        return 65 * L + c            # the transpose uses a row pitch of 65 words
    return cd * 64 + ((Ld + move_skew(move, cd)) & 63)


def move_read_word(move, L, c):
    if move == "T":
        return 65 * c + L
    return c * 64 + ((L + move_skew(move, c)) & 63)


@pytest.mark.parametrize("move", ["T", "RM2CM", "CM2RM"])
def test_layout_moves_are_the_intended_permutations(move):
    # whatever register c of lane L writes is read back by lane Ld as register cd
    written = {move_write_word(move, L, c): (L, c) for L in range(64) for c in range(64)}
    assert len(written) == 4096                      # no two writes share a word
    for L in range(64):
        for c in range(64):
            src = written[move_read_word(move, L, c)]
            assert move_dst(move, *src) == (L, c)
    if move != "T":
        # the super-row moves are inverse to each other and stay inside super-rows
        for L in range(64):
            for c in range(64):
                Ld, cd = move_dst(move, L, c)
                assert Ld >> 3 == L >> 3
                back = "CM2RM" if move == "RM2CM" else "RM2CM"
                assert move_dst(back, Ld, cd) == (L, c)


@pytest.mark.parametrize("move", ["T", "RM2CM", "CM2RM"])
@pytest.mark.parametrize("banks,phase", B32_MODELS)
def test_layout_moves_conflict_free(sim, move, banks, phase):
    model = sim.BankModel(banks, phase, 1)
    for c in range(64):   # one write and one read instruction per register
        w = [(L, move_write_word(move, L, c)) for L in range(64)]
        r = [(L, move_read_word(move, L, c)) for L in range(64)]
        assert sim.step_conflicts(w, model, is_read=False) == 0
        assert sim.step_conflicts(r, model, is_read=True) == 0


def test_unskewed_transpose_would_conflict(sim):
    # the same transpose with a row pitch of 64 puts a whole write on one bank
    model = sim.BankModel(32, 32, 1)
    w = [(L, 64 * L + 5) for L in range(64)]
    assert sim.step_conflicts(w, model, is_read=False) == 2 * 31


@pytest.mark.parametrize("m", [64, 128, 256])
def test_router_placement_conflict_free(sim, m):
    """Placement of the bank router: group g (4m slots) holds the items bound for
    destination class g (dst mod 16).  Lane l = 16q + g takes quarter q of group g: in
    step t it reads slot 4m g + q m + ((t + g + 16 q) mod m) (64-bit reads, 32-lane phases
    over 64 banks) and writes it to its destination, a slot congruent to g modulo 16
    (64-bit writes, 16-lane phases).  Over the m steps the four lanes of a group read
    each of its 4m slots exactly once."""
    rd = sim.BankModel(64, 32, 2)
    wr = sim.BankModel(64, 16, 2)
    rng = np.random.default_rng(m)
    seen = np.zeros(64 * m, dtype=int)
    for t in range(m):
        slots = [4 * m * (l % 16) + m * (l // 16) + ((t + l % 16 + 16 * (l // 16)) % m) for l in range(64)]
        for sl in slots:
            seen[sl] += 1
        assert sim.step_conflicts([(l, 2 * s) for l, s in enumerate(slots)], rd, is_read=True) == 0
        dst = [16 * int(rng.integers(0, 4 * m)) + l % 16 for l in range(64)]
        assert sim.step_conflicts([(l, 2 * s) for l, s in enumerate(dst)], wr, is_read=False) == 0
    assert (seen == 1).all()


def test_router_placement_needs_sixteen_classes(sim):
    """With eight classes lanes l and l + 8 of one 16-lane write phase carry the same
    class, and destinations 8 apart modulo 32 can meet: some write conflicts."""
    wr = sim.BankModel(64, 16, 2)
    dst = [32 * l + (l % 8) for l in range(64)]     # lanes l, l + 8: residues equal mod 32
    assert sim.step_conflicts([(l, 2 * s) for l, s in enumerate(dst)], wr, is_read=False) > 0


def test_router_class_splits_group_by_class():
    """Four MSD binary splits on the class bits (dst mod 16, top of the key) leave group
    g = slots [4m g, 4m (g + 1)) holding exactly the items of class g, for any
    permutation: the splits are stable partitions on the key's top four bits."""
    rng = np.random.default_rng(5)
    for n in (4096, 8192, 16384):
        dst = rng.permutation(n)
        key = ((dst % 16) << 28) | ((dst // 16) << 18) | np.arange(n)
        order = np.argsort(key >> 28, kind="stable")
        groups = (dst[order] % 16).reshape(16, n // 16)
        assert (groups == np.arange(16)[:, None]).all()
        # the key round-trips the destination and the source
        back = (((key >> 18) & 0x3FF) << 4) | (key >> 28)
        assert np.array_equal(back, dst) and np.array_equal(key & 0x3FFF, np.arange(n))


@pytest.mark.parametrize("banks,phase,width", [(32, 32, 1), (64, 32, 2), (64, 16, 2), (64, 64, 1)])
@pytest.mark.parametrize("is_read", [True, False])
def test_batch_conflicts_match_step_conflicts(sim, banks, phase, width, is_read):
    """The many-step count used for the counter predictions equals the one-step
    simulator on random address patterns (with repeated words and small ranges)."""
    from oracle import sim_predict
    rng = np.random.default_rng(banks + phase + width + is_read)
    model = sim.BankModel(banks, phase, width)
    for hi in (64, 200, 8192):
        words = rng.integers(0, hi, size=(40, 64)) * width
        got = sim_predict.batch_conflicts(words, model, is_read=is_read)
        want = [sim.step_conflicts(list(enumerate(w)), model, is_read=is_read) for w in words]
        assert list(got) == want


def test_naive_permute_prediction_closed_forms():
    """The transpose and bit-reversal families put all 32 lanes of a half on one bank
    (31 extra cycles per half, 62 per scattered instruction), the identity none."""
    from oracle import sim_predict
    n = 8192
    i = np.arange(n)
    transpose = (i % 64) * 128 + i // 64
    bitrev = np.array([int(f"{v:013b}"[::-1], 2) for v in range(n)])
    for pi in (transpose, bitrev):
        r = sim_predict.naive_permute_conflicts(pi, n, "scatter")
        assert r == {"instructions": 2 * n // 64, "conflict_cycles": 62 * n // 64}
    assert sim_predict.naive_permute_conflicts(i, n, "gather")["conflict_cycles"] == 0
