"""Pins of the CPU oracle against things other than itself.

Each test ties one oracle function to the mathematics: brute force over every
ordering / permutation of tiny tiles, library routines (Python ``sorted``,
numpy stable argsort, numpy transpose), closed forms, invariants and the
hand-worked fixtures in ``tests/golden/hand_worked.json``.  A few tests plant a
plausible mistake in a copy of an oracle result and check that the pins see it.
"""
import itertools
import json
import os

import numpy as np
import pytest

from paper_1507_01391_amd import inputs

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_worked.json")))


# ------------------------------------------------------------------------------------ helpers


def stable_order_by_definition(keys):
    """Ascending, ties by position -- via Python's built-in (stable) sorted()."""
    return sorted(range(len(keys)), key=lambda i: (keys[i], i))


def check_sort_invariants(keys, keys_out, perm):
    keys = np.asarray(keys)
    assert sorted(perm.tolist()) == list(range(len(keys))), "perm is not a permutation"
    assert np.array_equal(keys_out, keys[perm])
    assert np.all(keys_out[:-1] <= keys_out[1:])
    eq = keys_out[:-1] == keys_out[1:]
    assert np.all(perm[:-1][eq] < perm[1:][eq]), "equal keys not in input order"


# ---------------------------------------------------------------------------------- sorting


def test_sort_golden(oracle):
    g = GOLDEN["sort_stable"]
    k, p, perm = oracle.tile_sort(np.array(g["keys"], np.uint32), np.array(g["payload"], np.uint32))
    assert k.tolist() == g["keys_out"]
    assert perm.tolist() == g["perm"]
    assert p.tolist() == g["perm"]


@pytest.mark.parametrize("n", range(0, 7))
def test_sort_brute_force_all_orderings(oracle, n):
    """Every sequence over a 3-letter alphabet (duplicates included) for n <= 6."""
    if n == 0:
        k, _, perm = oracle.tile_sort(np.zeros(0, np.uint32))
        assert k.size == 0 and perm.size == 0
        return
    for seq in itertools.product((0, 7, 2**32 - 1), repeat=n):
        keys = np.array(seq, dtype=np.uint32)
        k, p, perm = oracle.tile_sort(keys, np.arange(n, dtype=np.uint32) + 100)
        want = stable_order_by_definition(seq)
        assert perm.tolist() == want
        assert (p - 100).tolist() == want
        check_sort_invariants(keys, k, perm)


def test_sort_matches_numpy_stable_argsort_multi_tile(oracle):
    rng = np.random.default_rng(11)
    sizes = rng.integers(0, 700, size=40)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    keys = rng.integers(0, 50, size=off[-1], dtype=np.uint32)  # many ties
    pay = rng.integers(0, 2**32, size=(3, off[-1]), dtype=np.uint32)
    k, p, perm = oracle.tile_sort(keys, pay, off)
    for t in range(len(sizes)):
        a, b = off[t], off[t + 1]
        order = np.argsort(keys[a:b], kind="stable")
        assert np.array_equal(perm[a:b], order)
        assert np.array_equal(k[a:b], keys[a:b][order])
        assert np.array_equal(p[:, a:b], pay[:, a:b][:, order])


def test_sort_f32_matches_float_order(oracle):
    rng = np.random.default_rng(5)
    special = np.array([-np.inf, -3.5, -1e-40, -0.0, 0.0, 1e-40, 2.5, np.inf, 1.0, -1.0],
                       dtype=np.float32)
    x = np.concatenate([rng.standard_normal(2000).astype(np.float32), special])
    rng.shuffle(x)
    k, _, perm = oracle.tile_sort(x, f32_ordered=True)
    # numpy orders -0.0 and +0.0 as equal; the bit map puts -0.0 first.  Compare on a
    # copy where -0.0 is replaced by the float just below +0.0's position in numpy.
    order = np.argsort(x, kind="stable")
    zeros = (x == 0)
    if zeros.sum() == 2:
        neg = np.where(zeros & np.signbit(x))[0][0]
        pos = np.where(zeros & ~np.signbit(x))[0][0]
        o = order.tolist()
        i, j = o.index(neg), o.index(pos)
        if i > j:
            o[i], o[j] = o[j], o[i]
        order = np.array(o)
    assert np.array_equal(perm, order)
    assert np.array_equal(k.view(np.uint32), x.view(np.uint32)[order])


def test_f32_order_golden_and_roundtrip(oracle):
    g = GOLDEN["f32_order"]
    bits = [int(b, 16) for b in g["bits"]]
    mapped = [int(b, 16) for b in g["mapped"]]
    for b, m in zip(bits, mapped):
        assert oracle.f32_order(b) == m
        assert oracle.f32_order_inv(m) == b
    assert mapped == sorted(mapped)  # the special values are listed in float order


def test_f32_order_monotone_random_pairs(oracle):
    rng = np.random.default_rng(3)
    a = rng.standard_normal(3000).astype(np.float32) * np.float32(1e3)
    b = rng.standard_normal(3000).astype(np.float32) * np.float32(1e-30)
    ua, ub = oracle.f32_order(a.view(np.uint32)), oracle.f32_order(b.view(np.uint32))
    assert np.array_equal(a < b, ua < ub)
    assert np.array_equal(oracle.f32_order_inv(ua), a.view(np.uint32))


def test_planted_unstable_sort_is_caught(oracle):
    """A plausible mistake -- swapping two equal keys' payloads -- breaks a pin."""
    keys = np.array([4, 1, 4, 4, 0], dtype=np.uint32)
    _, _, perm = oracle.tile_sort(keys)
    bad = perm.copy()
    i = int(np.where(keys[bad] == 4)[0][0])
    bad[i], bad[i + 1] = bad[i + 1], bad[i]
    with pytest.raises(AssertionError):
        check_sort_invariants(keys, keys[bad], bad)


# -------------------------------------------------------------------------------- partition


def test_partition_golden(oracle):
    g = GOLDEN["partition_w4"]
    lab, pay, perm = oracle.tile_partition(np.array(g["labels"]), np.array(g["payload"], np.uint32),
                                           num_classes=4)
    assert lab.tolist() == g["labels_out"]
    assert pay.tolist() == g["payload_out"]
    assert perm.tolist() == g["perm"]


@pytest.mark.parametrize("n", range(1, 7))
def test_partition_brute_force(oracle, n):
    for seq in itertools.product(range(3), repeat=n):
        lab = np.array(seq, dtype=np.uint32)
        out, _, perm = oracle.tile_partition(lab, num_classes=3)
        assert perm.tolist() == stable_order_by_definition(seq)
        assert out.tolist() == sorted(seq)


def test_partition_closed_form_exact_copies(oracle):
    """Exactly 64 copies of each class in a 4096-item tile: block c of the output is all c,
    and the items of a class keep their input order."""
    labels, payload, off = inputs.partition(seed=99, num_tiles=6)
    out, pay, perm = oracle.tile_partition(labels, payload.view(np.uint32), off)
    expect = np.tile(np.repeat(np.arange(64, dtype=np.uint32), 64), 6)
    assert np.array_equal(out, expect)
    for t in range(6):
        a = t * 4096
        p = perm[a:a + 4096].reshape(64, 64)
        assert np.all(np.diff(p, axis=1) > 0)
        assert np.array_equal(np.sort(p.reshape(-1)), np.arange(4096))
        assert np.array_equal(pay[a:a + 4096], payload.view(np.uint32)[a + perm[a:a + 4096]])


def test_partition_matches_numpy_uneven_classes(oracle):
    labels, payload, off = inputs.random_labels(seed=7, num_tiles=5, n=999, num_classes=17)
    out, pay, perm = oracle.tile_partition(labels, payload.view(np.uint32), off, num_classes=17)
    for t in range(5):
        a, b = off[t], off[t + 1]
        order = np.argsort(labels[a:b], kind="stable")
        assert np.array_equal(perm[a:b], order)
        assert np.array_equal(out[a:b], labels[a:b][order])


def test_partition_rejects_out_of_range_label(oracle):
    with pytest.raises(ValueError):
        oracle.tile_partition(np.array([0, 64, 1], np.uint32), num_classes=64)


# ------------------------------------------------------------------------------ permutation


def test_permute_golden(oracle):
    g = GOLDEN["permute"]
    x = np.array(g["x"], np.uint32)
    pi = np.array(g["pi"], np.int32)
    assert oracle.tile_permute(x, pi, oracle.SCATTER).tolist() == g["scatter"]
    assert oracle.tile_permute(x, pi, oracle.GATHER).tolist() == g["gather"]


@pytest.mark.parametrize("family", ["identity", "transpose", "bitrev"])
def test_permute_closed_forms(oracle, family):
    x, pi, _, off = inputs.permutation(seed=1, num_tiles=3, n=8192, family=family)
    out = oracle.tile_permute(x, pi, oracle.SCATTER, off)
    for t in range(3):
        xs = x[t * 8192:(t + 1) * 8192]
        os_ = out[t * 8192:(t + 1) * 8192]
        if family == "identity":
            want = xs
        elif family == "transpose":
            want = xs.reshape(128, 64).T.reshape(-1)      # numpy transpose
        else:
            idx = np.arange(8192)
            rev = np.array([int(format(i, "013b")[::-1], 2) for i in idx])
            want = xs[rev]                                 # bit reversal is an involution
        assert np.array_equal(os_.view(np.uint32), want.view(np.uint32))


def test_permute_gather_is_scatter_of_inverse_and_roundtrip(oracle):
    x, pi, _, off = inputs.permutation(seed=2, num_tiles=4, n=512, family="uniform")
    x2 = np.stack([x, -x])  # two channels, channel-planar
    inv = np.concatenate([np.argsort(pi[t * 512:(t + 1) * 512]) for t in range(4)]).astype(np.int32)
    g = oracle.tile_permute(x2, pi, oracle.GATHER, off)
    s_inv = oracle.tile_permute(x2, inv, oracle.SCATTER, off)
    assert np.array_equal(g.view(np.uint32), s_inv.view(np.uint32))
    back = oracle.tile_permute(oracle.tile_permute(x2, pi, oracle.SCATTER, off), pi, oracle.GATHER, off)
    assert np.array_equal(back.view(np.uint32), x2.view(np.uint32))
    # multiset of values is preserved per tile
    s = oracle.tile_permute(x, pi, oracle.SCATTER, off)
    for t in range(4):
        assert np.array_equal(np.sort(s[t * 512:(t + 1) * 512]), np.sort(x[t * 512:(t + 1) * 512]))


@pytest.mark.parametrize("n", range(1, 6))
def test_permute_brute_force_all_pi(oracle, n):
    x = (np.arange(n, dtype=np.uint32) * 37 + 5)
    for p in itertools.permutations(range(n)):
        pi = np.array(p, np.int32)
        s = oracle.tile_permute(x, pi, oracle.SCATTER)
        g = oracle.tile_permute(x, pi, oracle.GATHER)
        # compose with numpy fancy indexing (library) in both directions
        assert np.array_equal(s[pi], x)
        assert np.array_equal(g, x[pi])


def test_permute_rejects_non_permutation(oracle):
    with pytest.raises(ValueError):
        oracle.tile_permute(np.arange(4, dtype=np.uint32), np.array([0, 1, 1, 3], np.int32))
    with pytest.raises(ValueError):
        oracle.tile_permute(np.arange(4, dtype=np.uint32), np.array([0, 1, 2, 4], np.int32))
