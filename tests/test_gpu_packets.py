"""Served MC packets: the bytes a request is sent as decode to the stored MC voxels, and
with the cut-off plus zstd they take less than a tenth of the TSDF packets of the same
blocks (the bandwidth saving claimed in Sec. 6.2 and the bandwidth table)."""
import numpy as np
import pytest

from datagen import configs
from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


def test_mc_packets_decode_and_save_bandwidth():
    vbh = require_gpu()
    from paper_1805_03709_amd import packets
    _, depth, rgb, poses = configs.tiny_inputs(32)
    S = vbh.Scene(vbh.make_params(configs.TINY_VOL, configs.TINY_CAM))
    for f in range(32):
        S.vbh_integrate_frame(depth[f].cuda(), rgb[f].cuda(), poses[f], f + 1)
    assert S.vbh_scene_status() == 0
    cursor, mc_bytes, tsdf_bytes, blocks = 0, 0, 0, 0
    while True:
        keys, meta = S.vbh_updated_blocks_since(cursor, 512)
        cnt, cursor = (int(v) for v in meta.tolist())
        if cnt == 0:
            break
        kk = keys[:cnt].contiguous()
        mc, c3 = S.vbh_stored_mc(kk)
        mc, c3 = mc.cpu().numpy().astype(np.uint32), c3.cpu().numpy().astype(np.uint32)
        packed = mc | (c3[..., 0] << 8) | (c3[..., 1] << 16) | (c3[..., 2] << 24)
        raw = packets.mc_packet(kk.cpu().numpy(), packed)
        z = packets.zstd_compress(raw)
        back = np.frombuffer(packets.zstd_decompress(z, len(raw)), np.uint8).reshape(cnt, -1)
        assert np.array_equal(back[:, :12].copy().view("<i4"), kk.cpu().numpy())
        assert np.array_equal(back[:, 12:].copy().view("<u4"), packed)
        # cut-off: indices 0 and 255 carry no colour
        idx = packed & 0xFF
        assert ((packed[(idx == 0) | (idx == 255)]) == 0).all()
        F, W, c, found = S.vbh_scene_read_blocks(kk)
        assert bool(found.all())
        tz = packets.zstd_compress(packets.tsdf_packet(kk.cpu().numpy(), F.cpu().numpy(), W.cpu().numpy(),
                                                       c.cpu().numpy()))
        mc_bytes, tsdf_bytes, blocks = mc_bytes + len(z), tsdf_bytes + len(tz), blocks + cnt
    assert blocks == S.vbh_scene_stats()["n_blocks"]
    say(f"[packets] {blocks} blocks: MC {mc_bytes / blocks:.1f} B/block, TSDF {tsdf_bytes / blocks:.1f} B/block "
        f"compressed ({100 * (1 - mc_bytes / tsdf_bytes):.1f} % saved)")
    assert mc_bytes < 0.1 * tsdf_bytes
