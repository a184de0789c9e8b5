"""Pins of the oracle's scene reset (Sec. 4.1, quasi-static scenes) and of its selection
of the currently visible blocks: a float64 frustum test written independently, set
algebra over the update set and the log, and the identity "reset everything, fuse the
same frames again" == "fuse them into a fresh volume"."""
import dataclasses

import numpy as np

from datagen import configs

VOL = dataclasses.replace(configs.TINY_VOL, depth_min=0.3, depth_max=1.1)
CAM = configs.TINY_CAM


def fused(orc, n, vol=VOL, first=0, ids=None):
    _, depth, rgb, poses = configs.tiny_inputs(max(n + first, 21))
    S = orc.Scene(vol, CAM)
    for i, f in enumerate(range(first, first + n)):
        assert S.integrate(depth[f].numpy(), rgb[f].numpy(), poses[f], (ids or (lambda j: j + 1))(i)) == 0
    return S, depth, rgb, poses


def visible64(keys, pose, vol=VOL, cam=CAM):
    """float64 frustum test of each block's central voxel (local 4,4,4); also returns which
    blocks are far (1e-4 px, 1e-6 m) from every decision boundary."""
    vs = float(np.float32(vol.voxel_size))
    R, t = pose[:, :3].astype(np.float64), pose[:, 3].astype(np.float64)
    p = (keys.astype(np.float64) * 8 + 4) * vs
    pc = (p - t) @ R  # R^T (p - t), row by row
    z = pc[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = cam.fx * (pc[:, 0] / z) + cam.cx + 0.5
        v = cam.fy * (pc[:, 1] / z) + cam.cy + 0.5
    inside = (z > 0) & (z >= vol.depth_min) & (z <= vol.depth_max) & (np.floor(u) >= 0) & (np.floor(u) < cam.width) \
        & (np.floor(v) >= 0) & (np.floor(v) < cam.height)
    safe = (np.abs(u - np.round(u)) > 1e-4) & (np.abs(v - np.round(v)) > 1e-4) & \
        (np.abs(z - vol.depth_min) > 1e-6) & (np.abs(z - vol.depth_max) > 1e-6)
    return inside, safe


def test_visible_blocks_match_float64_frustum(orc):
    S, _, _, poses = fused(orc, 6)
    keys = S.blocks()
    assert keys.shape[0] > 200
    gated = 0
    for f in (0, 3, 5, 7, 12, 20):
        got = {tuple(k) for k in S.visible_blocks(poses[f])}
        inside, safe = visible64(keys, poses[f])
        want = {tuple(k) for k in keys[inside & safe]}
        gs = {tuple(k) for k in keys[safe]}
        assert got & gs == want, f
        assert got <= {tuple(k) for k in keys}
        # some but not all blocks are visible, and the depth range removes some of them
        assert 0 < len(want) < keys.shape[0]
        wide = dataclasses.replace(VOL, depth_min=0.0, depth_max=float("inf"))
        inside_w, _ = visible64(keys, poses[f], vol=wide)
        gated += int((inside_w & ~inside).sum())
    assert gated > 0


def test_reset_clears_logs_and_republishes(orc):
    S, _, _, poses = fused(orc, 6)
    keys_all = S.blocks()
    F0, W0, C0, _ = S.read(keys_all)
    mc0, _ = S.stored_mc(keys_all)
    vis = S.visible_blocks(poses[2])
    absent = np.array([[900, 900, 900], [-900, 5, 5]], np.int32)
    req = np.concatenate([vis, vis[:5], absent])
    mark = S.log_length()
    n_before = S.n_blocks()
    rc, n_reset = S.reset_blocks(req, 7)
    assert rc == 0 and n_reset == vis.shape[0]
    assert S.n_blocks() == n_before  # nothing allocated
    assert {tuple(k) for k in S.last_touched()} == {tuple(k) for k in vis}
    F1, W1, C1, _ = S.read(keys_all)
    isr = np.array([tuple(k) in {tuple(v) for v in vis} for k in keys_all])
    assert (W1[isr] == 0).all() and (F1[isr] == 0).all() and (C1[isr] == 0).all()
    assert np.array_equal(F1[~isr], F0[~isr]) and np.array_equal(W1[~isr], W0[~isr])
    assert np.array_equal(C1[~isr], C0[~isr])
    # update set: the reset blocks and their existing negative neighbours
    have = {tuple(k) for k in keys_all}
    want = set()
    for k in vis:
        for e in range(8):
            n = (k[0] - (e & 1), k[1] - ((e >> 1) & 1), k[2] - ((e >> 2) & 1))
            if n in have:
                want.add(n)
    upd = {tuple(k) for k in S.last_mc_updated()}
    assert upd == want
    assert S.log_length() - mark == len(want)
    got, _ = S.updated_since(mark, 1 << 30)
    assert {tuple(k) for k in got} == want
    # MC voxels: reset blocks carry nothing; every refreshed block equals a fresh extraction;
    # blocks outside the update set keep their stored voxels
    mc1, rgb1 = S.stored_mc(keys_all)
    assert (mc1[isr] == 0).all() and (rgb1[isr] == 0).all()
    inset = np.array([tuple(k) in want for k in keys_all])
    fresh, _ = S.extract_mc(keys_all[inset])
    assert np.array_equal(mc1[inset], fresh)
    assert np.array_equal(mc1[~inset], mc0[~inset])
    assert (mc0[isr] != 0).any()  # the reset really removed surface
    # frame ids must still increase; an empty reset is a valid (empty) update
    assert S.reset_blocks(vis, 7)[0] != 0
    assert S.reset_blocks(absent, 8) == (0, 0) and S.last_mc_updated().shape[0] == 0


def test_reset_everything_then_refuse_equals_fresh_volume(orc):
    A, depth, rgb, poses = fused(orc, 4)
    assert A.reset_blocks(A.blocks(), 5) == (0, A.n_blocks())
    for i in range(4):
        assert A.integrate(depth[i].numpy(), rgb[i].numpy(), poses[i], 6 + i) == 0
    B, _, _, _ = fused(orc, 4)
    kb = B.blocks()
    Fa, Wa, Ca, fa = A.read(kb)
    Fb, Wb, Cb, _ = B.read(kb)
    assert fa.all()
    assert np.array_equal(Fa, Fb) and np.array_equal(Wa, Wb) and np.array_equal(Ca, Cb)
    # blocks only in A were reset and never observed again
    extra = np.array([k for k in A.blocks() if tuple(k) not in {tuple(x) for x in kb}], np.int32).reshape(-1, 3)
    if extra.shape[0]:
        assert (A.read(extra)[1] == 0).all()
    assert np.array_equal(A.extract_mc(kb)[0], B.extract_mc(kb)[0])
