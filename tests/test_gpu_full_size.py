"""Parity at the full workload sizes, in the launch configuration bench.py times, on
outputs the oracle computes tile by tile (a sample of tiles / segments / rows)."""
import numpy as np
import pytest
import torch

from paper_1507_01391_amd import inputs

pytestmark = pytest.mark.gpu

SAMPLE = 12


@pytest.fixture(scope="module")
def ts():
    import paper_1507_01391_amd as ts
    return ts


def sample(count, seed):
    return np.sort(np.random.default_rng(seed).choice(count, size=min(SAMPLE, count), replace=False))


def test_c2_partition_65536_tiles(ts, oracle):
    labels, payload, off = inputs.partition(num_tiles=65536)
    dl = torch.from_numpy(labels.view(np.int32)).cuda()
    dp = torch.from_numpy(payload).cuda()
    lo, po, _ = ts.tile_partition(dl, dp, torch.from_numpy(off).cuda(), 64, max_tile_len=4096)
    ts.check_device_errors()
    lh, ph = lo.cpu().numpy().view(np.uint32), po.cpu().numpy().view(np.uint32)
    del dl, dp, lo, po
    for t in list(sample(65536, 1)) + [0, 65535]:
        a, b = int(off[t]), int(off[t + 1])
        wl, wp, _ = oracle.tile_partition(labels[a:b], payload[a:b].view(np.uint32), num_classes=64)
        assert np.array_equal(lh[a:b], wl) and np.array_equal(ph[a:b], wp), t
    # every tile: exactly 64 copies of each class, in class order
    assert np.array_equal(lh.reshape(65536, 4096), np.broadcast_to(np.repeat(np.arange(64, dtype=np.uint32), 64), (65536, 4096)))


def test_c3_permute_fwd_bwd_16384_tiles(ts, oracle):
    x, pi, g, off = inputs.permutation(num_tiles=16384, n=8192)
    dx, dpi = torch.from_numpy(x).cuda(), torch.from_numpy(pi).cuda()
    dg, doff = torch.from_numpy(g).cuda(), torch.from_numpy(off).cuda()
    inv = torch.empty_like(dpi)
    y = ts.tile_permute(dx, dpi, "scatter", doff, max_tile_len=8192, inv_out=inv)
    gx = ts.tile_permute(dg, inv, "scatter", doff, max_tile_len=8192)
    ts.check_device_errors()
    yh, gh, ih = y.cpu().numpy(), gx.cpu().numpy(), inv.cpu().numpy()
    del dx, dpi, dg, y, gx, inv
    for t in sample(16384, 2):
        a, b = int(off[t]), int(off[t + 1])
        wy = oracle.tile_permute(x[a:b].view(np.uint32), pi[a:b], oracle.SCATTER)
        wg = oracle.tile_permute(g[a:b].view(np.uint32), pi[a:b], oracle.GATHER)
        assert np.array_equal(yh[a:b].view(np.uint32), wy), t
        assert np.array_equal(gh[a:b].view(np.uint32), wg), t
        assert np.array_equal(ih[a:b][pi[a:b]], np.arange(b - a, dtype=np.int32)), t


def test_c4_segments_100000_graph(ts, oracle):
    keys, payload, off, kinds = inputs.segments(num_segments=100000)
    dk = torch.from_numpy(keys.view(np.int32)).cuda()
    dp = torch.from_numpy(payload.view(np.int32)).cuda()
    g = ts.sort_graph(dk, torch.from_numpy(off).cuda(), 32768, payload=dp)
    g.replay()
    torch.cuda.synchronize()
    ts.check_device_errors()
    ko, po, pm = g.result
    kh, ph, mh = ko.cpu().numpy().view(np.uint32), po.cpu().numpy().view(np.uint32), pm.cpu().numpy()
    del g, dk, dp, ko, po, pm
    sizes = np.diff(off)
    picks = list(sample(100000, 3)) + [int(np.argmax(sizes)), int(np.argmin(sizes))]
    for kind in range(len(inputs.SEGMENT_KINDS)):           # one of every key distribution
        picks.append(int(np.nonzero(kinds == kind)[0][0]))
    for s in picks:
        a, b = int(off[s]), int(off[s + 1])
        wk, wp, wperm = oracle.tile_sort(keys[a:b], payload[a:b])
        assert np.array_equal(kh[a:b], wk) and np.array_equal(ph[a:b], wp), s
        assert np.array_equal(mh[a:b], wperm), s


def test_c5_sort_with_payload_4096_rows(ts):
    keys, payload, grad, off = inputs.sort_payload(rows=4096)
    dk = torch.from_numpy(keys).cuda().requires_grad_(True)
    dp = torch.from_numpy(payload).cuda().requires_grad_(True)
    gk = torch.from_numpy(np.random.default_rng(5).standard_normal(keys.shape[0], dtype=np.float32)).cuda()
    sk, sp, perm = ts.sort_with_payload(dk, dp, torch.from_numpy(off).cuda(), 16384)
    torch.autograd.backward([sk, sp], [gk, torch.from_numpy(grad).cuda()])
    skh, sph, permh = sk.detach().cpu().numpy(), sp.detach().cpu().numpy(), perm.cpu().numpy()
    gkh, gph = dk.grad.cpu().numpy(), dp.grad.cpu().numpy()
    gk_h = gk.cpu().numpy()
    n = 16384
    for r in sample(4096, 4):
        a, b = r * n, (r + 1) * n
        idx = np.argsort(keys[a:b], kind="stable")        # N(0,1) keys: no +-0 or NaN
        assert np.array_equal(permh[a:b], idx.astype(np.int32)), r
        assert np.array_equal(skh[a:b].view(np.uint32), keys[a:b][idx].view(np.uint32)), r
        assert np.array_equal(sph[:, a:b].view(np.uint32), payload[:, a:b][:, idx].view(np.uint32)), r
        want_gp = np.empty_like(payload[:, a:b])
        want_gp[:, idx] = grad[:, a:b]
        want_gk = np.empty(n, np.float32)
        want_gk[idx] = gk_h[a:b]
        assert np.array_equal(gph[:, a:b].view(np.uint32), want_gp.view(np.uint32)), r
        assert np.array_equal(gkh[a:b].view(np.uint32), want_gk.view(np.uint32)), r
