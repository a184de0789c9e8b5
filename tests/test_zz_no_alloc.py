"""The allocation-free triangulation entry point (vbh_mc_triangulate_static) against
vbh_mc_triangulate with a caller workspace, through the C ABI: two calls in a row on the
same device, the second with fewer blocks (the static workspace keeps the first call's
contents), then a request beyond the stated maximum."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_util import require_gpu, say, to_dev
from test_oracle_mesh import mc_blocks

pytestmark = pytest.mark.gpu


def sphere_blocks(r, lo, hi):
    vs, c = 0.01, np.array([0.0031, -0.0017, 0.0043])
    sdf = lambda p: np.linalg.norm(p - c, axis=-1) - r
    keys, mcv = mc_blocks(sdf, np.array(lo), np.array(hi), vs)
    return to_dev(keys), to_dev(mcv.view(np.int32)), vs


def run(lib, fn, keys, mcv, vs, cap, work=None):
    n = keys.shape[0]
    pos = torch.full((max(cap, 1), 3, 3), -7.0, device="cuda")
    rgb = torch.full((max(cap, 1), 3), 7, dtype=torch.uint8, device="cuda")
    cnt = C.c_int64(-1)
    args = [C.c_void_p(keys.data_ptr()), C.c_void_p(mcv.data_ptr()), n, C.c_float(vs),
            C.c_void_p(pos.data_ptr()), C.c_void_p(rgb.data_ptr()), cap]
    if work is not None:
        args.append(C.c_void_p(work.data_ptr()))
    rc = getattr(lib, fn)(*args, C.byref(cnt), None)
    torch.cuda.synchronize()
    return rc, cnt.value, pos.cpu().numpy(), rgb.cpu().numpy()


def test_static_workspace_equals_caller_workspace():
    vbh = require_gpu()
    lib = vbh.lib()
    for r, lo, hi in ((0.25, [-32] * 3, [32] * 3), (0.1037, [-14] * 3, [14] * 3)):
        keys, mcv, vs = sphere_blocks(r, lo, hi)
        n = keys.shape[0]
        work = torch.empty(int(lib.vbh_mc_work_size(n)), dtype=torch.int64, device="cuda")
        rc0, c0, _, _ = run(lib, "vbh_mc_triangulate", keys, mcv, vs, 0, work)  # count only
        assert rc0 == 0 and c0 > 0
        rc1, c1, p1, g1 = run(lib, "vbh_mc_triangulate", keys, mcv, vs, c0, work)
        rc2, c2, p2, g2 = run(lib, "vbh_mc_triangulate_static", keys, mcv, vs, c0)
        say(f"[no-alloc] {n} blocks, {c2} triangles")
        assert rc1 == 0 and rc2 == 0 and c1 == c2 == c0
        assert np.array_equal(p1, p2) and np.array_equal(g1, g2)
        # a short output buffer: the leading triangles, the full count
        rc3, c3, p3, _ = run(lib, "vbh_mc_triangulate_static", keys, mcv, vs, 100)
        assert rc3 == 0 and c3 == c0 and np.array_equal(p3[:100], p1[:100])
    # beyond the stated maximum: an error, nothing enqueued
    big = lib.vbh_mc_triangulate_static(C.c_void_p(keys.data_ptr()), C.c_void_p(mcv.data_ptr()), (1 << 20) + 1,
                                        C.c_float(vs), None, None, 0, C.byref(C.c_int64()), None)
    assert big == vbh.binding.VBH_EINVAL
