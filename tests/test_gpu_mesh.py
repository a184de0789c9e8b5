"""GPU client triangulation (Sec. 4.3) against the oracle, triangle for triangle: on MC
voxels built from an analytic sphere, on the MC voxels of the fused tiny scene (several
scan chunks and a ragged tail), with a short output buffer and with no blocks; and the
fused scene's mesh against the analytic surface it was rendered from."""
import numpy as np
import pytest
import torch

from datagen import configs
from datagen.scenes import scene_sdf
from gpu_util import require_gpu, say, to_dev
from test_oracle_mesh import mc_blocks, mesh_checks

pytestmark = pytest.mark.gpu


def test_sphere_equals_oracle(orc):
    vbh = require_gpu()
    vs, r, c = 0.01, 0.1037, np.array([0.0031, -0.0017, 0.0043])
    sdf = lambda p: np.linalg.norm(p - c, axis=-1) - r
    keys, mcv = mc_blocks(sdf, np.array([-14, -14, -14]), np.array([14, 14, 14]), vs)
    pos, rgb = vbh.vbh_mc_triangulate(to_dev(keys), to_dev(mcv.view(np.int32)), vs)
    opos, orgb = orc.mc_triangles(keys, mcv, vs)
    say(f"[mesh sphere] {pos.shape[0]} triangles")
    assert pos.shape == torch.Size(opos.shape)
    assert np.array_equal(pos.cpu().numpy(), opos) and np.array_equal(rgb.cpu().numpy(), orgb)
    chi, _ = mesh_checks(pos.cpu().numpy(), vs, sdf)
    assert chi == 2


def test_fused_scene_equals_oracle_and_follows_the_surface(orc):
    vbh = require_gpu()
    scene, depth, rgb, poses = configs.tiny_inputs(32)
    S = vbh.Scene(vbh.make_params(configs.TINY_VOL, configs.TINY_CAM))
    for f in range(32):
        S.vbh_integrate_frame(depth[f].cuda(), rgb[f].cuda(), poses[f], f + 1)
    keys = S.vbh_scene_export_blocks()
    mc, c3 = S.vbh_stored_mc(keys)
    mcv = (mc.to(torch.int64) | c3[..., 0].to(torch.int64) << 8 | c3[..., 1].to(torch.int64) << 16
           | c3[..., 2].to(torch.int64) << 24).to(torch.uint32).view(torch.int32).contiguous()
    n = keys.shape[0]
    assert n > 3 * 1024  # several scan chunks, ragged tail
    pos, col = vbh.vbh_mc_triangulate(keys, mcv, configs.TINY_VOL.voxel_size)
    opos, ocol = orc.mc_triangles(keys.cpu().numpy(), mcv.cpu().numpy().view(np.uint32), configs.TINY_VOL.voxel_size)
    say(f"[mesh tiny] {n} blocks, {pos.shape[0]} triangles")
    assert np.array_equal(pos.cpu().numpy(), opos) and np.array_equal(col.cpu().numpy(), ocol)
    # against the analytic surface the frames were rendered from (noise-free depth)
    v = torch.as_tensor(opos.reshape(-1, 3), dtype=torch.float64)
    d = scene_sdf(scene, v).abs().numpy() / configs.TINY_VOL.voxel_size
    q = np.quantile(d, [0.5, 0.99])
    say(f"[mesh tiny] |sdf| at vertices in voxels: median {q[0]:.3f}, p99 {q[1]:.3f}, max {d.max():.3f}")
    assert q[0] <= 0.5 and q[1] <= 1.0
    # a short buffer gets the first triangles; no blocks give no triangles
    k = 1000
    work = torch.empty(int(vbh.lib().vbh_mc_work_size(n)), dtype=torch.int64, device="cuda")
    buf = torch.full((k, 3, 3), -7.0, device="cuda")
    import ctypes as C
    cnt = C.c_int64()
    rc = vbh.lib().vbh_mc_triangulate(C.c_void_p(keys.data_ptr()), C.c_void_p(mcv.data_ptr()), n,
                                      configs.TINY_VOL.voxel_size, C.c_void_p(buf.data_ptr()), None, k,
                                      C.c_void_p(work.data_ptr()), C.byref(cnt), None)
    torch.cuda.synchronize()
    assert rc == 0 and cnt.value == opos.shape[0]
    assert np.array_equal(buf.cpu().numpy(), opos[:k])
    e_pos, _ = vbh.vbh_mc_triangulate(keys[:0], mcv[:0], configs.TINY_VOL.voxel_size)
    assert e_pos.shape[0] == 0
