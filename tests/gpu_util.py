"""Helpers shared by the GPU parity tests."""
import sys

import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1805_03709_amd as vbh
    vbh.lib()  # raises if the library is not built: no fallback
    return vbh


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def keyset(keys) -> set:
    k = keys.cpu().numpy() if isinstance(keys, torch.Tensor) else np.asarray(keys)
    return set(map(tuple, k.reshape(-1, 3).tolist()))


def sort_keys(keys):
    k = np.asarray(keys).reshape(-1, 3)
    order = np.lexsort((k[:, 2], k[:, 1], k[:, 0]))
    return k[order], order


CORNERS = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)])


def corner_min_abs(O, keys, blk, loc):
    """min over the 8 cell corners of |F_oracle| for the voxels (keys[blk], local loc),
    read from oracle scene O in one call (absent or unobserved corners read as 0)."""
    blk, loc = np.asarray(blk), np.asarray(loc)
    if blk.size == 0:
        return np.zeros(0)
    g = keys[blk].astype(np.int64) * 8 + np.stack([loc % 8, (loc // 8) % 8, loc // 64], -1)
    cs = g[:, None, :] + CORNERS[None]                      # [m, 8, 3]
    B = np.floor_divide(cs, 8)
    uniq, inv = np.unique(B.reshape(-1, 3), axis=0, return_inverse=True)
    F, _, _, _ = O.read(uniq.astype(np.int32))
    lc = cs - 8 * B
    li = (lc[..., 0] + 8 * lc[..., 1] + 64 * lc[..., 2]).reshape(-1)
    return np.abs(F[inv.reshape(-1), li]).reshape(-1, 8).min(axis=1)


def pack_mc(mc, rgb):
    """uint8 index [.., 512] and RGB [.., 512, 3] -> the 4-byte MC voxel as int64."""
    m = torch.as_tensor(mc).to(torch.int64)
    c = torch.as_tensor(rgb).to(torch.int64)
    return m | c[..., 0] << 8 | c[..., 1] << 16 | c[..., 2] << 24
