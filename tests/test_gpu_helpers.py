"""GPU checks of the measurement helpers: the HBM reference copy (the denominator of
the copy-bandwidth figure) and the LDS access probe (the bank model)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ts():
    import paper_1507_01391_amd as ts
    return ts


@pytest.mark.parametrize("nbytes", [5, 16, 48, 32768 - 16, 32768, 32768 + 16, 1000003, 1000016, (1 << 24) + 4096 + 16])
@pytest.mark.parametrize("offset", [0, 16, 4096 + 48])
def test_copy_bit_exact(ts, nbytes, offset):
    """Odd sizes (the bytes past the last 16-byte multiple take the tail kernel), starts
    16-byte aligned: exactly the bytes asked for are copied, the bytes after them are
    untouched."""
    rng = np.random.default_rng(nbytes + offset)
    total = offset + nbytes + 4096
    src_h = rng.integers(0, 256, size=total, dtype=np.uint8)
    src = torch.from_numpy(src_h).cuda()
    dst = torch.zeros(total, dtype=torch.uint8, device="cuda")
    ts.copy(src[offset:offset + nbytes], dst[offset:offset + nbytes + 4096])
    torch.cuda.synchronize()
    got = dst.cpu().numpy()
    assert np.array_equal(got[offset:offset + nbytes], src_h[offset:offset + nbytes])
    assert not got[:offset].any() and not got[offset + nbytes:].any()


def test_copy_rejects_misaligned(ts):
    from paper_1507_01391_amd._lib import TileSortError
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(TileSortError, match="aligned"):
        ts.copy(buf[4:1028], buf[2048:3072])


def test_lds_probe_counts_and_sink(ts):
    """One probe per access kind: every wave reports a positive cycle count, and a read
    probe returns the words it read (the probe fills its LDS array with the word index
    before the timed loop, so the sink holds lane_words)."""
    lanes = list(range(64))
    for op, width in (("read", 1), ("read", 2), ("write", 1), ("bpermute", 1)):
        cycles, sink = ts.lds_probe(lanes, op=op, width=width, iters=64, waves=2, groups=3)
        torch.cuda.synchronize()
        assert cycles.numel() == 6 and bool((cycles > 0).all()), (op, width)
        assert sink.numel() == 6 * 64
