"""The boundary's generic forms: vbh_size (live keys), vbh_status on either kind of handle,
and vbh_extract_mc_all (the extraction of every allocated block), against the specific
calls they stand for."""
import numpy as np
import pytest
import torch

from datagen import configs
from gpu_util import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu
ABSENT = -(1 << 31)


def test_size_and_status_on_maps():
    vbh = require_gpu()
    for m in (vbh.Map(1 << 10, 0), vbh.ChainedMap(256, 256, 1)):
        keys = np.stack(np.meshgrid(np.arange(6), np.arange(5), np.arange(4), indexing="ij"), -1).reshape(-1, 3)
        keys = keys.astype(np.int32)
        m.vbh_insert(to_dev(keys), to_dev(np.arange(len(keys), dtype=np.int32)))
        m.vbh_erase(to_dev(keys[:17]))
        assert m.vbh_size() == m.vbh_map_size()[0] == len(keys) - 17
        assert m.vbh_status() == 0
        # a sticky error read through the generic call, then cleared
        m.vbh_insert(to_dev(np.array([[1, 2, 3]], np.int32)), to_dev(np.array([ABSENT], np.int32)))
        assert m.vbh_status() == vbh.binding.VBH_EINVAL
        assert m.vbh_status() == 0 and m.vbh_map_status() == 0


def test_status_on_scene_and_rejects_null():
    vbh = require_gpu()
    _, depth, rgb, poses = configs.tiny_inputs(4)
    S = vbh.Scene(vbh.make_params(configs.TINY_VOL, configs.TINY_CAM))
    S.vbh_integrate_frame(depth[0].cuda(), rgb[0].cuda(), poses[0], 1)
    assert S.vbh_status() == 0
    # keys out of range written through the ABI record VBH_EINVAL on the scene
    bad = torch.tensor([[1 << 20, 0, 0]], dtype=torch.int32, device="cuda")
    S.vbh_scene_write_blocks(bad, torch.zeros((1, 512), device="cuda"), torch.ones((1, 512), dtype=torch.uint8,
                             device="cuda"), None, 2)
    assert S.vbh_status() == vbh.binding.VBH_EINVAL
    assert S.vbh_status() == 0 and S.vbh_scene_status() == 0
    assert vbh.binding.lib().vbh_status(None, None) == vbh.binding.VBH_EINVAL


def test_extract_mc_all_equals_per_key_extraction():
    vbh = require_gpu()
    _, depth, rgb, poses = configs.tiny_inputs(12)
    S = vbh.Scene(vbh.make_params(configs.TINY_VOL, configs.TINY_CAM))
    for f in range(12):
        S.vbh_integrate_frame(depth[f].cuda(), rgb[f].cuda(), poses[f], f + 1)
    keys_ref = S.vbh_scene_export_blocks()
    n = keys_ref.shape[0]
    say(f"[api forms] {n} blocks")
    assert n > 100
    keys, mc, rgb_out, total = S.vbh_extract_mc_all(n + 10)
    assert total == n and keys.shape[0] == n
    assert torch.equal(keys, keys_ref)
    mc_ref, rgb_ref = S.vbh_extract_mc_indices(keys_ref)
    assert torch.equal(mc, mc_ref) and torch.equal(rgb_out, rgb_ref)
    # a smaller capacity: the first cap blocks, and the full count
    keys2, mc2, _, total2 = S.vbh_extract_mc_all(n // 3, with_rgb=False)
    assert total2 == n and keys2.shape[0] == n // 3
    assert torch.equal(keys2, keys_ref[: n // 3]) and torch.equal(mc2, mc_ref[: n // 3])
    assert S.vbh_status() == 0
