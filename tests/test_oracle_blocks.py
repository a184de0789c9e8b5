"""Pins of the oracle's explicit-block-list fusion (integration into given blocks instead
of the band blocks).

- Given exactly the band blocks of a frame, it equals the band fusion of that frame:
  state, touched/new/MC sets and the update log.
- A fronto-parallel wall at depth D seen head-on: every listed block between the camera
  and the wall has each voxel that projects into the image at a lattice point z < D - mu
  observed once with F = mu (the clamp), and voxels behind the wall by more than mu stay
  unobserved; colour equals the observed colour.
"""
import numpy as np

import oracle
from datagen import configs
from datagen.configs import Volume
from datagen.scenes import Camera


def test_band_blocks_reproduce_band_fusion(orc):
    _, depth, rgb, poses = configs.tiny_inputs(4)
    A = orc.Scene(configs.TINY_VOL, configs.TINY_CAM)
    B = orc.Scene(configs.TINY_VOL, configs.TINY_CAM)
    for f in range(3):
        assert A.integrate(depth[f].numpy(), rgb[f].numpy(), poses[f], f + 1) == 0
        band = A.last_touched()
        # shuffled, with duplicates
        rng = np.random.default_rng(f)
        lst = np.concatenate([band, band[rng.integers(0, band.shape[0], 50)]])[rng.permutation(band.shape[0] + 50)]
        assert B.integrate_blocks(lst, depth[f].numpy(), rgb[f].numpy(), poses[f], f + 1) == 0
        for fn in ("last_touched", "last_new", "last_mc_updated"):
            assert np.array_equal(getattr(A, fn)(), getattr(B, fn)()), fn
    keys = A.blocks()
    for x, y in zip(A.read(keys), B.read(keys)):
        assert np.array_equal(x, y)
    assert np.array_equal(A.stored_mc(keys)[0], B.stored_mc(keys)[0])
    assert A.log_length() == B.log_length()
    ka, _ = A.updated_since(0, 1 << 20)
    kb, _ = B.updated_since(0, 1 << 20)
    assert np.array_equal(ka, kb)


def test_fronto_parallel_wall():
    vs, mu, D = 0.01, 0.04, 1.5
    vol = Volume(slots=1 << 16, pool_blocks=1 << 14, voxel_size=vs, trunc=mu, depth_min=0.0,
                 depth_max=float("inf"), log_capacity=1 << 20)
    cam = Camera(64, 48, 40.0, 40.0, 31.5, 23.5)
    O = oracle.Scene(vol, cam)
    depth = np.full((cam.height, cam.width), D, np.float32)
    rgb = np.zeros((cam.height, cam.width, 3), np.uint8)
    rgb[..., 0], rgb[..., 1], rgb[..., 2] = 10, 20, 30
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])  # camera at the origin looking along +z
    keys = np.array([(x, y, z) for x in range(-4, 4) for y in range(-3, 3) for z in range(1, 22)], np.int32)
    assert O.integrate_blocks(keys, depth, rgb, pose, 1) == 0
    assert O.last_new().shape[0] == keys.shape[0]
    F, W, c, found = O.read(keys)
    assert found.all()
    l = np.arange(512)
    g = keys[:, None, :].astype(np.int64) * 8 + np.stack([l % 8, (l // 8) % 8, l // 64], -1)[None]
    X = g * vs
    z = X[..., 2]
    u = np.floor(cam.fx * (X[..., 0] / np.maximum(z, 1e-9)) + cam.cx + 0.5)
    v = np.floor(cam.fy * (X[..., 1] / np.maximum(z, 1e-9)) + cam.cy + 0.5)
    inside = (z > 0) & (u >= 0) & (u < cam.width) & (v >= 0) & (v < cam.height)
    # decisions away from float32 ties: margins on the pixel and on the truncation edges
    fu = cam.fx * (X[..., 0] / np.maximum(z, 1e-9)) + cam.cx + 0.5
    fv = cam.fy * (X[..., 1] / np.maximum(z, 1e-9)) + cam.cy + 0.5
    clear = (np.abs(fu - np.round(fu)) > 1e-3) & (np.abs(fv - np.round(fv)) > 1e-3)
    front = inside & clear & (z < D - mu - 1e-4)
    behind = inside & clear & (z > D + mu + 1e-4)
    band = inside & clear & (z > D - mu + 1e-4) & (z < D + mu - 1e-4)
    assert front.sum() > 10000 and behind.sum() > 1000 and band.sum() > 1000
    assert (W[front] == 1).all() and np.allclose(F[front], mu, atol=1e-12)
    assert (c[front] == [10, 20, 30]).all()
    assert (W[behind] == 0).all()
    assert (W[band] == 1).all() and np.allclose(F[band], D - z[band], atol=1e-6)
    assert (W[~inside] == 0).all()
