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
