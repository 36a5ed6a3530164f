"""Differentiable sort-with-payload and permutation (torch.autograd.Function).

Both backward passes move the upstream gradient through the inverse of the
forward permutation with the same conflict-free tile kernels; indices and keys
stay exact integers throughout.

* ``Permute``:  y = scatter(x, pi), i.e. y[pi[i]] = x[i]; dx[i] = dy[pi[i]], computed as
  a scatter by pi^-1, which the forward routing writes out at no extra pass (a direct
  gather would route twice).
* ``SortWithPayload``: keys are fp32, sorted ascending through the order-preserving
  bit map (stable; -0 before +0); payload_out[:, k] = payload[:, perm[k]] and
  sorted_keys[k] = keys[perm[k]]; backward scatters: dp[:, perm[k]] = dpo[:, k], and
  the key gradient the same way, both by one routing per tile (the key gradient rides
  as an extra channel of the payload gradient's scatter).
"""
from __future__ import annotations

import torch

from . import ops

# Longest tile the backward scatter (tile_permute) moves.
PERMUTE_MAX_TILE = 16384


def _resolve_max_len(offsets, max_tile_len):
    """max_tile_len, or the longest tile of `offsets` read once (one device sync) when it
    is not given; passing it keeps forward and backward free of host synchronisation."""
    ml = ops.longest_tile(offsets) if max_tile_len is None else int(max_tile_len)
    if ml > PERMUTE_MAX_TILE:
        raise ValueError(f"tiles of up to {PERMUTE_MAX_TILE} items are differentiable "
                         f"(the backward scatter's capacity); got max_tile_len {ml}")
    return ml


class Permute(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, pi, offsets, max_tile_len=None):
        max_tile_len = _resolve_max_len(offsets, max_tile_len)
        # the inverse is kept as 16-bit tile-local indices (every supported tile
        # length fits), so the backward reads 2 bytes per element for it
        inv = torch.empty(pi.shape, dtype=torch.int16, device=pi.device)
        y = ops.tile_permute(x.contiguous(), pi, "scatter", offsets, max_tile_len, inv_out=inv)
        ctx.save_for_backward(inv, offsets)
        ctx.max_tile_len = max_tile_len
        return y

    @staticmethod
    def backward(ctx, gy):
        inv, offsets = ctx.saved_tensors
        gx = ops.tile_permute(gy.contiguous(), inv, "scatter", offsets, ctx.max_tile_len)
        return gx, None, None, None


class SortWithPayload(torch.autograd.Function):
    @staticmethod
    def forward(ctx, keys, payload, offsets, max_tile_len=None):
        assert keys.dtype == torch.float32, "keys must be float32"
        max_tile_len = _resolve_max_len(offsets, max_tile_len)
        k, p, perm = ops.tile_sort(keys.contiguous(), payload.contiguous(), offsets,
                                   max_tile_len=max_tile_len, f32_ordered=True, want_perm=True)
        ctx.save_for_backward(perm, offsets)
        ctx.max_tile_len = max_tile_len
        ctx.mark_non_differentiable(perm)
        # gradients of outputs that the loss does not use arrive as None instead of
        # being materialised as zero tensors (the permutation's would be a 4 B/key fill)
        ctx.set_materialize_grads(False)
        return k, p, perm

    @staticmethod
    def backward(ctx, g_keys, g_payload, g_perm):
        perm, offsets = ctx.saved_tensors
        want_k = g_keys is not None and ctx.needs_input_grad[0]
        want_p = g_payload is not None and ctx.needs_input_grad[1]
        gk = gp = None
        if want_k and want_p:
            # one routing per tile moves both: the key gradient as the extra channel
            gp, gk = ops.tile_permute(g_payload.contiguous(), perm, "scatter", offsets, ctx.max_tile_len,
                                      aux=g_keys.contiguous())
        elif want_k:
            gk = ops.tile_permute(g_keys.contiguous(), perm, "scatter", offsets, ctx.max_tile_len)
        elif want_p:
            gp = ops.tile_permute(g_payload.contiguous(), perm, "scatter", offsets, ctx.max_tile_len)
        return gk, gp, None, None


def permute(x, pi, offsets, max_tile_len=None):
    return Permute.apply(x, pi, offsets, max_tile_len)


def sort_with_payload(keys, payload, offsets, max_tile_len=None):
    return SortWithPayload.apply(keys, payload, offsets, max_tile_len)
