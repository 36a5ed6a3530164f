"""Helpers for the GPU parity tests: numpy <-> device transfers of 32-bit words."""
import numpy as np
import torch


def dev(a):
    """numpy array of 32/64-bit values -> GPU tensor with the same bits."""
    a = np.ascontiguousarray(a)
    if a.dtype in (np.uint32, np.float32):
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def host_u32(t):
    return t.cpu().numpy().view(np.uint32)


def host_i32(t):
    return t.cpu().numpy().view(np.int32)
