"""GPU parity of allocation, integration, MC voxels and the update log against the oracle.

Bar: key sets, allocation sets, W and colour bit-exact; F within 1e-5 m of the float64
oracle; MC voxels bit-exact on identical F/W input, and end to end only where some
corner has |F_oracle| <= 1e-5.
"""
import math

import numpy as np
import pytest
import torch

from datagen import configs
from gpu_util import corner_min_abs, keyset, require_gpu, say, sort_keys, to_dev

pytestmark = pytest.mark.gpu
F_TOL = 1e-5


def pose_np(p):
    return np.asarray(p, np.float64).reshape(3, 4)


def make_pair(vbh, orc, vol, cam, hash_kind=0):
    return vbh.Scene(vbh.make_params(vol, cam, hash_kind)), orc.Scene(vol, cam)


def integrate_both(G, O, depth, rgb, poses, frames, first_id=1, check_frames=True):
    for i, f in enumerate(frames):
        fid = first_id + i
        d, c = depth[f], rgb[f]
        G.vbh_integrate_frame(to_dev(d.numpy() if torch.is_tensor(d) else d),
                              to_dev(c.numpy() if torch.is_tensor(c) else c), poses[f], fid)
        rc = O.integrate(d.numpy() if torch.is_tensor(d) else d, c.numpy() if torch.is_tensor(c) else c,
                         poses[f], fid)
        assert rc == 0
        if check_frames:
            st = G.vbh_scene_stats()
            gt = keyset(G.vbh_scene_last_touched())
            ot = keyset(O.last_touched())
            say(f"  frame {fid}: touched {len(gt)} new {st['n_new']} mc {st['n_mc']}")
            assert gt == ot, (len(gt), len(ot), len(gt ^ ot))
            assert st["n_touched"] == len(ot) and st["n_new"] == len(O.last_new())
            assert keyset(G.vbh_scene_last_mc()) == keyset(O.last_mc_updated())
    assert G.vbh_scene_status() == 0


def compare_state(G, O):
    gk = G.vbh_scene_export_blocks().cpu().numpy()
    ok = O.blocks()
    assert keyset(gk) == keyset(ok) and gk.shape[0] == ok.shape[0]
    keys, _ = sort_keys(ok)
    dk = to_dev(keys)
    F, W, rgb, found = (t.cpu().numpy() for t in G.vbh_scene_read_blocks(dk))
    oF, oW, orgb, ofound = O.read(keys)
    assert found.all() and ofound.all()
    assert np.array_equal(W, oW)
    assert np.array_equal(rgb, orgb)
    err = np.abs(F.astype(np.float64) - oF)
    say(f"  blocks {keys.shape[0]}  max|F-F64| {err.max():.3g}  observed {(W > 0).sum()}")
    assert err.max() <= F_TOL
    # MC voxels, end to end: differences only where a corner's F is within 1e-5 of 0
    gmc, grgb = (t.cpu().numpy() for t in G.vbh_stored_mc(dk))
    omc, orgb2 = O.stored_mc(keys)
    mism = np.nonzero(gmc != omc)
    say(f"  MC end-to-end mismatches: {mism[0].size}")
    if mism[0].size:
        assert (corner_min_abs(O, keys, *mism) <= F_TOL).all()
    return keys, F, W, rgb, gmc, grgb


def mc_on_identical_input(orc, vol, cam, keys, F, W, rgb, gmc, grgb):
    O2 = orc.Scene(vol, cam)
    assert O2.write(keys, F, W, rgb, 1) == 0
    omc, orgb = O2.extract_mc(keys)
    assert np.array_equal(gmc, omc)
    assert np.array_equal(grgb, orgb)


def test_tiny_full_pipeline(orc):
    """32 noise-free 320x240 frames around the box room, 1 cm voxels, then MC of every block."""
    vbh = require_gpu()
    say("[scene tiny] generating")
    _, depth, rgb, poses = configs.tiny_inputs(32)
    G, O = make_pair(vbh, orc, configs.TINY_VOL, configs.TINY_CAM)
    integrate_both(G, O, depth, rgb, poses, range(32))
    keys, F, W, rgb_, gmc, grgb = compare_state(G, O)
    mc_on_identical_input(orc, configs.TINY_VOL, configs.TINY_CAM, keys, F, W, rgb_, gmc, grgb)
    # on-demand extraction equals the MC pool kept up to date frame by frame
    emc, ergb = G.vbh_extract_mc_indices(to_dev(keys))
    assert np.array_equal(emc.cpu().numpy(), gmc) and np.array_equal(ergb.cpu().numpy(), grgb)
    assert (gmc > 0).sum() > 10000


@pytest.mark.parametrize("hash_kind", [0, 1])
def test_full_size_frames(orc, hash_kind):
    """First frames of the 640x480 noisy sequence at 5 mm voxels in the full-size volume and
    launch configuration (2^22 slots, 2^21-block pool)."""
    vbh = require_gpu()
    n = 6 if hash_kind == 0 else 3
    say(f"[scene full] hash={hash_kind} generating {n} frames")
    _, depth, rgb, poses = configs.full_inputs(range(n))
    G, O = make_pair(vbh, orc, configs.FULL_VOL, configs.FULL_CAM, hash_kind)
    integrate_both(G, O, depth, rgb, poses, range(n))
    keys, F, W, rgb_, gmc, grgb = compare_state(G, O)
    mc_on_identical_input(orc, configs.FULL_VOL, configs.FULL_CAM, keys, F, W, rgb_, gmc, grgb)


def test_mc_identical_input_sphere_and_edges(orc):
    vbh = require_gpu()
    rng = np.random.default_rng(3)
    keys = np.array([(x, y, z) for x in range(-1, 3) for y in range(-1, 2) for z in range(0, 3)], np.int32)
    keys = keys[rng.permutation(keys.shape[0])[:30]]  # some neighbours missing
    loc = np.arange(512)
    l3 = np.stack([loc % 8, (loc // 8) % 8, loc // 64], -1)
    g = keys[:, None, :].astype(np.int64) * 8 + l3[None]
    F = (np.linalg.norm(g - np.array([4.3, 5.1, 9.7]), axis=-1) - 7.2).astype(np.float32) * 0.01
    W = np.where(rng.random(F.shape) < 0.01, 0, rng.integers(1, 256, size=F.shape)).astype(np.uint8)
    rgb = rng.integers(0, 256, size=F.shape + (3,)).astype(np.uint8)
    G = vbh.Scene(vbh.make_params(configs.TINY_VOL, configs.TINY_CAM))
    G.vbh_scene_write_blocks(to_dev(keys), to_dev(F), to_dev(W), to_dev(rgb), 1)
    O = orc.Scene(configs.TINY_VOL, configs.TINY_CAM)
    O.write(keys, F, W, rgb, 1)
    q = np.concatenate([keys, np.array([[50, 50, 50]], np.int32)])  # plus a missing block
    gmc, grgb = (t.cpu().numpy() for t in G.vbh_extract_mc_indices(to_dev(q)))
    omc, orgb = O.extract_mc(q)
    assert np.array_equal(gmc, omc) and np.array_equal(grgb, orgb)
    assert (gmc[-1] == 0).all() and (gmc > 0).sum() > 100
    smc, srgb = (t.cpu().numpy() for t in G.vbh_stored_mc(to_dev(q)))
    assert np.array_equal(smc, omc) and np.array_equal(srgb, orgb)
    # read-back of the written state
    Fr, Wr, rgbr, found = (t.cpu().numpy() for t in G.vbh_scene_read_blocks(to_dev(q)))
    assert np.array_equal(Fr[:-1], F) and np.array_equal(Wr[:-1], W) and np.array_equal(rgbr[:-1], rgb)
    assert found[:-1].all() and found[-1] == 0


def test_updated_since_against_oracle(orc):
    vbh = require_gpu()
    _, depth, rgb, poses = configs.tiny_inputs(8)
    G, O = make_pair(vbh, orc, configs.TINY_VOL, configs.TINY_CAM)
    marks = []
    for f in range(8):
        marks.append(O.log_length())
        integrate_both(G, O, depth, rgb, poses, [f], first_id=f + 1, check_frames=False)
    assert G.vbh_scene_stats()["log_length"] == O.log_length()
    for cur in [0] + marks[1:] + [O.log_length(), O.log_length() + 5]:
        keys, meta = G.vbh_updated_blocks_since(cur, 1 << 20)
        n, nxt = (int(x) for x in meta.cpu())
        ok, onxt = O.updated_since(cur, 1 << 20)
        assert keyset(keys[:n]) == keyset(ok) and n == ok.shape[0]
        assert nxt == onxt
    # pages: union = everything, no duplicates, cursors advance
    cur, seen = 0, []
    while True:
        keys, meta = G.vbh_updated_blocks_since(cur, 333)
        n, nxt = (int(x) for x in meta.cpu())
        seen += [tuple(k) for k in keys[:n].cpu().numpy()]
        if n < 333:
            assert nxt == O.log_length()
            break
        assert nxt > cur
        cur = nxt
    assert len(seen) == len(set(seen)) and set(seen) == keyset(O.blocks())
    keys, meta = G.vbh_updated_blocks_since(7, 0)
    assert [int(x) for x in meta.cpu()] == [0, 7]


def test_scene_errors(orc):
    vbh = require_gpu()
    _, depth, rgb, poses = configs.tiny_inputs(2)
    G = vbh.Scene(vbh.make_params(configs.TINY_VOL, configs.TINY_CAM))
    G.vbh_integrate_frame(to_dev(depth[0].numpy()), None, poses[0], 5)
    with pytest.raises(vbh.VbhError):
        G.vbh_integrate_frame(to_dev(depth[1].numpy()), None, poses[1], 5)
    small = configs.Volume(**{**configs.TINY_VOL.__dict__, "pool_blocks": 100})
    G2 = vbh.Scene(vbh.make_params(small, configs.TINY_CAM))
    G2.vbh_integrate_frame(to_dev(depth[0].numpy()), None, poses[0], 1)
    assert G2.vbh_scene_status() == vbh.binding.VBH_EFULL_POOL
    assert G2.vbh_scene_stats()["n_blocks"] == 100
    G2.vbh_integrate_frame(to_dev(depth[1].numpy()), None, poses[1], 2)  # still runs, still reports
    assert G2.vbh_scene_status() == vbh.binding.VBH_EFULL_POOL
    tiny_log = configs.Volume(**{**configs.TINY_VOL.__dict__, "log_capacity": 10})
    G3 = vbh.Scene(vbh.make_params(tiny_log, configs.TINY_CAM))
    G3.vbh_integrate_frame(to_dev(depth[0].numpy()), None, poses[0], 1)
    assert G3.vbh_scene_status() == vbh.binding.VBH_EFULL_LOG


def test_ragged_empty_and_invalid_frames(orc):
    """A 101x77 camera (no dimension a multiple of the 32x16 allocation tile or the 8x8
    wave tile), an all-zero frame, a frame whose depths all lie outside [dmin, dmax], and a
    frame fused on top of blocks written through the ABI: touched/new/MC sets, state and MC
    voxels against the oracle after every frame."""
    vbh = require_gpu()
    cam = configs.Camera(101, 77, 90.0, 90.0, 50.0, 38.0)
    vol = configs.Volume(**{**configs.TINY_VOL.__dict__, "depth_min": 0.3, "depth_max": 3.0})
    _, depth, rgb, poses = configs.tiny_inputs(6, cam=cam)
    depth, rgb = depth.numpy().copy(), rgb.numpy().copy()
    depth[2] = 0.0                                   # every pixel invalid
    depth[3] = np.where(depth[3] > 0, 3.5, 0.0)      # every depth beyond dmax
    G, O = make_pair(vbh, orc, vol, cam)
    integrate_both(G, O, depth, rgb, poses, range(2))
    for f in (2, 3):
        integrate_both(G, O, depth, rgb, poses, [f], first_id=f + 1)
        st = G.vbh_scene_stats()
        assert st["n_touched"] == 0 and st["n_new"] == 0 and st["n_mc"] == 0
    # overwrite some blocks (sign words rebuilt from the written voxels), then fuse on top
    keys, _ = sort_keys(O.blocks())
    sel = keys[::3]
    rng = np.random.default_rng(7)
    F = rng.normal(0.0, 0.02, (sel.shape[0], 512)).astype(np.float32)
    W = np.where(rng.random(F.shape) < 0.2, 0, rng.integers(1, 200, size=F.shape)).astype(np.uint8)
    c = rng.integers(0, 256, size=F.shape + (3,)).astype(np.uint8)
    G.vbh_scene_write_blocks(to_dev(sel), to_dev(F), to_dev(W), to_dev(c), 5)
    assert O.write(sel, F, W, c, 5) == 0
    integrate_both(G, O, depth, rgb, poses, [4, 5], first_id=6)
    k2, F2, W2, rgb2, gmc, grgb = compare_state(G, O)
    mc_on_identical_input(orc, vol, cam, k2, F2, W2, rgb2, gmc, grgb)
    emc, ergb = G.vbh_extract_mc_indices(to_dev(k2))
    assert np.array_equal(emc.cpu().numpy(), gmc) and np.array_equal(ergb.cpu().numpy(), grgb)


def test_world_scaled_by_power_of_two_takes_full_divisions(orc):
    """Every length (voxel size, truncation, depths, translations) multiplied by 2^30.
    Scaling by a power of two commutes with float rounding, so the scene must come out
    identical to the unscaled one (keys, W, colour and MC voxels bit-exact, F scaled
    exactly by 2^30).  At this scale the host's coordinate bounds exceed 2^32, so
    integration projects with the full float division and the float pixel test (the
    unscaled scene takes the reciprocal-based quotient and the integer test), and
    allocation divides fully in both (the tiny volume has no finite depth_max).  The scaled
    scene is also checked against the oracle."""
    vbh = require_gpu()
    S = 2.0 ** 30
    _, depth, rgb, poses = configs.tiny_inputs(6)
    vol = configs.TINY_VOL
    vol_s = configs.Volume(**{**vol.__dict__, "voxel_size": vol.voxel_size * S, "trunc": vol.trunc * S})
    poses_s = poses.copy()
    poses_s[..., 3] *= S
    depth_s = depth * S
    G, O = make_pair(vbh, orc, vol, configs.TINY_CAM)
    Gs, Os = make_pair(vbh, orc, vol_s, configs.TINY_CAM)
    integrate_both(G, O, depth, rgb, poses, range(6), check_frames=False)
    integrate_both(Gs, Os, depth_s, rgb, poses_s, range(6))
    keys, _ = sort_keys(G.vbh_scene_export_blocks().cpu().numpy())
    assert keyset(keys) == keyset(Gs.vbh_scene_export_blocks())
    dk = to_dev(keys)
    F, W, c, _ = (t.cpu().numpy() for t in G.vbh_scene_read_blocks(dk))
    Fs, Ws, cs, _ = (t.cpu().numpy() for t in Gs.vbh_scene_read_blocks(dk))
    assert np.array_equal(W, Ws) and np.array_equal(c, cs)
    assert np.array_equal(F * np.float32(S), Fs)
    for x, y in zip(G.vbh_stored_mc(dk), Gs.vbh_stored_mc(dk)):
        assert torch.equal(x, y)
    st, sts = G.vbh_scene_stats(), Gs.vbh_scene_stats()
    assert st["total_voxel_updates"] == sts["total_voxel_updates"] and st["log_length"] == sts["log_length"]
    # against the oracle fed the scaled inputs (F within the scaled tolerance)
    ok = Os.blocks()
    assert keyset(ok) == keyset(keys)
    oF, oW, orgb, _ = Os.read(keys)
    assert np.array_equal(Ws, oW) and np.array_equal(cs, orgb)
    err = np.abs(Fs.astype(np.float64) - oF).max()
    say(f"  {keys.shape[0]} blocks, max|F-F64| {err:.3g} at scale 2^30")
    assert err <= F_TOL * S


def test_zero_world_coordinates_take_the_full_division(orc):
    """A camera with identity rotation at (0, 0, -0.95) and a principal point on a pixel
    centre: band samples on the principal column (row) have world x (y) exactly 0, below
    the range of the reciprocal-based quotient, so their waves take the full division in
    allocation; a finite depth range keeps the reciprocal path on for the others.  Sets
    and state against the oracle over two frames (the second revisits every block)."""
    vbh = require_gpu()
    from datagen.scenes import render_frames
    cam = configs.Camera(101, 77, 90.0, 90.0, 50.0, 38.0)
    vol = configs.Volume(**{**configs.TINY_VOL.__dict__, "depth_min": 0.3, "depth_max": 3.0})
    scene, _, _, _ = configs.tiny_inputs(1)
    pose = np.array([[1.0, 0.0, 0.0, 0.0], [0.0, 1.0, 0.0, 0.0], [0.0, 0.0, 1.0, -0.95]])
    depth, rgb = render_frames(scene, cam, [pose, pose])
    dn = depth.numpy()
    assert ((dn[0] >= 0.3) & (dn[0] <= 3.0)).mean() > 0.5
    assert dn[0, 38, 50] > 0.3 and dn[0, 20, 50] > 0.3 and dn[0, 38, 20] > 0.3
    G, O = make_pair(vbh, orc, vol, cam)
    integrate_both(G, O, depth, rgb, [pose, pose], range(2))
    k2, F2, W2, rgb2, gmc, grgb = compare_state(G, O)
    assert (W2 == 2).any()
    mc_on_identical_input(orc, vol, cam, k2, F2, W2, rgb2, gmc, grgb)


def test_local_keys_at_both_ends_of_their_range(orc):
    """Allocation's 32-bit local keys hold each block coordinate as an offset in [0, 1024)
    from a base 512 blocks below the camera's block.  Here 0.5 mm voxels (4 mm blocks), a
    2 m depth limit and a narrow camera put the host's reach at 510 blocks, just inside the
    511 it admits, and two views of the far walls 1.95 m away (along +z, then along -z)
    give z offsets near 999 and near 25.  Sets and state against the oracle."""
    vbh = require_gpu()
    from datagen.scenes import render_frames
    cam = configs.Camera(101, 77, 2000.0, 2000.0, 50.0, 38.0)
    vol = configs.Volume(slots=1 << 16, pool_blocks=1 << 14, voxel_size=0.0005, trunc=0.002,
                         depth_min=0.3, depth_max=2.0, log_capacity=1 << 20)
    # the host's bound (camera depth at most dmax + mu + 2 m vs + vs, identity-like rows)
    lam = vol.depth_max + vol.trunc + 2 * 4 * vol.voxel_size + vol.voxel_size
    reach = math.ceil((1.01 * lam + 2.0 ** -20 * 1.95) / (8 * vol.voxel_size)) + 3
    assert 500 <= reach <= 511
    scene, _, _, _ = configs.tiny_inputs(1)
    poses = np.array([[[1.0, 0.0, 0.0, 0.85], [0.0, 1.0, 0.0, 0.85], [0.0, 0.0, 1.0, -0.95]],
                      [[-1.0, 0.0, 0.0, 0.85], [0.0, 1.0, 0.0, 0.85], [0.0, 0.0, -1.0, 0.95]]])
    depth, rgb = render_frames(scene, cam, poses)
    assert ((depth.numpy() > 1.9) & (depth.numpy() < 2.0)).all()
    G, O = make_pair(vbh, orc, vol, cam)
    integrate_both(G, O, depth, rgb, poses, range(2))
    keys = O.blocks()
    bz = keys[:, 2].astype(np.int64)
    say(f"  block z from {bz.min()} to {bz.max()} (camera blocks {int(np.floor(-0.95 / 0.004))}, {int(np.floor(0.95 / 0.004))})")
    assert bz.max() - int(np.floor(-0.95 / 0.004)) >= 480 and int(np.floor(0.95 / 0.004)) - bz.min() >= 480
    k2, F2, W2, rgb2, gmc, grgb = compare_state(G, O)
    mc_on_identical_input(orc, vol, cam, k2, F2, W2, rgb2, gmc, grgb)


def same_scene(A, B):
    """Bit-exact equality of two scenes: statistics, last touched/MC sets, block set, voxel
    state, MC voxels and the update log (a multiset per frame, frames in order)."""
    sa, sb = A.vbh_scene_stats(), B.vbh_scene_stats()
    for k in ("n_blocks", "log_length", "total_touched", "total_mc", "total_voxel_updates", "n_touched", "n_mc"):
        assert sa[k] == sb[k], k
    assert keyset(A.vbh_scene_last_touched()) == keyset(B.vbh_scene_last_touched())
    assert keyset(A.vbh_scene_last_mc()) == keyset(B.vbh_scene_last_mc())
    keys, _ = sort_keys(A.vbh_scene_export_blocks().cpu().numpy())
    assert keyset(keys) == keyset(B.vbh_scene_export_blocks())
    dk = to_dev(keys)
    for x, y in zip(A.vbh_scene_read_blocks(dk), B.vbh_scene_read_blocks(dk)):
        assert torch.equal(x, y)
    for x, y in zip(A.vbh_stored_mc(dk), B.vbh_stored_mc(dk)):
        assert torch.equal(x, y)
    L = sa["log_length"]
    la = [t.cpu().numpy() for t in A.vbh_scene_log_entries(0, L)]
    lb = [t.cpu().numpy() for t in B.vbh_scene_log_entries(0, L)]
    ra = sorted(zip(la[0].tolist(), map(tuple, la[1].tolist())))
    rb = sorted(zip(lb[0].tolist(), map(tuple, lb[1].tolist())))
    assert ra == rb and (np.diff(lb[0]) >= 0).all()
    say(f"  {keys.shape[0]} blocks, {L} log entries identical")


def test_multi_frame_form_equals_per_frame_calls(orc):
    """vbh_integrate_frames against one vbh_integrate_frame call per frame, on the full-size volume:
    block set, voxel state, MC voxels, update log and statistics bit-exact; then the
    multi-frame scene against the oracle."""
    vbh = require_gpu()
    n = 10
    say(f"[scene multi-frame] generating {n} full-size frames")
    _, depth, rgb, poses = configs.full_inputs(range(n))
    d, c = depth.cuda(), rgb.cuda()
    params = vbh.make_params(configs.FULL_VOL, configs.FULL_CAM)
    A, B = vbh.Scene(params), vbh.Scene(params)
    per_frame = []
    for f in range(n):
        A.vbh_integrate_frame(d[f], c[f], poses[f], f + 1)
        st = A.vbh_scene_stats()
        per_frame.append((st["n_touched"], st["n_mc"]))
    B.vbh_scene_enable_timing(2)
    B.vbh_integrate_frames(d[:4].contiguous(), c[:4].contiguous(), poses[:4], 1)
    B.vbh_integrate_frames(d[4:].contiguous(), c[4:].contiguous(), poses[4:], 5)
    assert A.vbh_scene_status() == 0 and B.vbh_scene_status() == 0
    ms, timed, blocks = B.vbh_scene_timing(with_blocks=True)
    assert timed == n // 2 and ms["alloc"] > 0 and ms["integrate"] > 0 and ms["mc_extract"] > 0
    # the block counts of exactly the timed updates (every second one, from the first)
    assert blocks == tuple(int(sum(x[i] for x in per_frame[::2])) for i in range(2))
    assert B.vbh_scene_timing(with_blocks=True)[1:] == (0, (0, 0))  # reset by the read
    same_scene(A, B)
    with pytest.raises(vbh.VbhError):
        B.vbh_integrate_frames(d[:1].contiguous(), c[:1].contiguous(), poses[:1], n)  # id not increasing
    # and the multi-frame form against the oracle
    O = orc.Scene(configs.FULL_VOL, configs.FULL_CAM)
    for f in range(n):
        assert O.integrate(depth[f].numpy(), rgb[f].numpy(), poses[f], f + 1) == 0
    compare_state(B, O)


def test_host_input_frames_equal_device_input():
    """vbh_integrate_frames_host (frames in pinned host memory, uploaded into two device
    buffers in front of each frame's kernels), split over two calls, against
    vbh_integrate_frames on device copies of the same frames: bit-exact."""
    vbh = require_gpu()
    n = 7
    say(f"[scene host input] generating {n} full-size frames")
    _, depth, rgb, poses = configs.full_inputs(range(n))
    params = vbh.make_params(configs.FULL_VOL, configs.FULL_CAM)
    A, B = vbh.Scene(params), vbh.Scene(params)
    A.vbh_integrate_frames(depth.cuda(), rgb.cuda(), poses, 1)
    hd, hc = depth.contiguous().pin_memory(), rgb.contiguous().pin_memory()
    B.vbh_integrate_frames_host(hd[:3], hc[:3], poses[:3], 1)
    B.vbh_integrate_frames_host(hd[3:], hc[3:], poses[3:], 4)
    torch.cuda.synchronize()
    assert A.vbh_scene_status() == 0 and B.vbh_scene_status() == 0
    same_scene(A, B)
    with pytest.raises(TypeError):
        B.vbh_integrate_frames_host(depth[:1].cuda(), None, poses[:1], n + 1)  # device tensor refused


def test_saturated_weights(orc):
    """Blocks written with W in {254, 255} (and a few 0 and 253), mixed colours and F, then
    three frames fused on top: the running mean at saturation (n = 256, W stays 255) for F
    and colour, W and RGB bit-exact and F within 1e-5 m of the oracle."""
    vbh = require_gpu()
    _, depth, rgb, poses = configs.tiny_inputs(8)
    G, O = make_pair(vbh, orc, configs.TINY_VOL, configs.TINY_CAM)
    integrate_both(G, O, depth, rgb, poses, range(2))
    keys, _ = sort_keys(O.blocks())
    rng = np.random.default_rng(255)
    F = rng.uniform(-0.04, 0.04, (keys.shape[0], 512)).astype(np.float32)
    W = rng.choice(np.array([0, 253, 254, 255, 255, 255], np.uint8), size=F.shape)
    c = rng.integers(0, 256, size=F.shape + (3,)).astype(np.uint8)
    G.vbh_scene_write_blocks(to_dev(keys), to_dev(F), to_dev(W), to_dev(c), 3)
    assert O.write(keys, F, W, c, 3) == 0
    integrate_both(G, O, depth, rgb, poses, [2, 3, 4], first_id=4)
    k2, F2, W2, rgb2, gmc, grgb = compare_state(G, O)
    # the saturation branch was taken: voxels written at 255 that were observed again
    pos = {tuple(k): i for i, k in enumerate(k2.tolist())}
    idx = np.array([pos[tuple(k)] for k in keys.tolist()])
    sat = (W == 255) & ((F2[idx] != F) | np.any(rgb2[idx] != c, axis=-1))
    from254 = (W == 254) & (W2[idx] == 255)
    say(f"  saturated voxels updated: {sat.sum()}, 254 -> 255: {from254.sum()}")
    assert sat.sum() > 1000 and from254.sum() > 100
    assert (W2[idx][W == 255] == 255).all()
    mc_on_identical_input(orc, configs.TINY_VOL, configs.TINY_CAM, k2, F2, W2, rgb2, gmc, grgb)


def test_full_size_long_run(orc):
    """150 frames of the 640x480 noisy sequence at 5 mm voxels in the full-size volume:
    touched, new and MC sets bit-exact on every 10th frame, then the whole final state
    (revisited blocks, weights up to the frame count) against the oracle."""
    vbh = require_gpu()
    n = 150
    say(f"[scene full long] generating {n} frames")
    _, depth, rgb, poses = configs.full_inputs(range(n), device="cuda")
    depth, rgb = depth.contiguous(), rgb.contiguous()
    hd, hc = depth.cpu().numpy(), rgb.cpu().numpy()
    G, O = make_pair(vbh, orc, configs.FULL_VOL, configs.FULL_CAM)
    for f in range(n):
        G.vbh_integrate_frame(depth[f], rgb[f], poses[f], f + 1)
        assert O.integrate(hd[f], hc[f], poses[f], f + 1) == 0
        if f % 10 == 9:
            st = G.vbh_scene_stats()
            gt, ot = keyset(G.vbh_scene_last_touched()), keyset(O.last_touched())
            assert gt == ot, (f, len(gt), len(ot))
            assert st["n_new"] == len(O.last_new())
            assert keyset(G.vbh_scene_last_mc()) == keyset(O.last_mc_updated())
            say(f"  frame {f + 1}: touched {len(gt)} new {st['n_new']} blocks {st['n_blocks']}")
    assert G.vbh_scene_status() == 0
    keys, F, W, rgb_, gmc, grgb = compare_state(G, O)
    say(f"  max W {W.max()}")
    assert W.max() >= 100
    mc_on_identical_input(orc, configs.FULL_VOL, configs.FULL_CAM, keys, F, W, rgb_, gmc, grgb)


def test_integrate_blocks_against_oracle(orc):
    """Integration of a frame into an explicit block list (the band blocks of that frame,
    a slab of blocks across the room that are mostly new and partly in free space, and
    duplicates), then a band-fused frame on top: touched, new and MC sets, state and MC
    voxels against the oracle."""
    vbh = require_gpu()
    _, depth, rgb, poses = configs.tiny_inputs(8)
    G, O = make_pair(vbh, orc, configs.TINY_VOL, configs.TINY_CAM)
    integrate_both(G, O, depth, rgb, poses, range(3))
    scratch = orc.Scene(configs.TINY_VOL, configs.TINY_CAM)
    assert scratch.integrate(depth[3].numpy(), rgb[3].numpy(), poses[3], 1) == 0
    band = scratch.last_touched()
    slab = np.array([(x, y, z) for x in range(-13, 13) for y in range(-13, 13) for z in range(-2, 2)], np.int32)
    rng = np.random.default_rng(11)
    lst = np.concatenate([band, slab, band[rng.integers(0, band.shape[0], 200)]])
    lst = lst[rng.permutation(lst.shape[0])]
    G.vbh_integrate_blocks(to_dev(lst), to_dev(depth[3].numpy()), to_dev(rgb[3].numpy()), poses[3], 4)
    assert O.integrate_blocks(lst, depth[3].numpy(), rgb[3].numpy(), poses[3], 4) == 0
    st = G.vbh_scene_stats()
    say(f"  listed {lst.shape[0]} keys: touched {st['n_touched']} new {st['n_new']} mc {st['n_mc']}")
    assert keyset(G.vbh_scene_last_touched()) == keyset(O.last_touched())
    assert st["n_touched"] == O.last_touched().shape[0] and st["n_new"] == O.last_new().shape[0]
    assert keyset(G.vbh_scene_last_mc()) == keyset(O.last_mc_updated())
    assert G.vbh_scene_status() == 0
    integrate_both(G, O, depth, rgb, poses, [4], first_id=5)
    keys, F, W, rgb_, gmc, grgb = compare_state(G, O)
    mc_on_identical_input(orc, configs.TINY_VOL, configs.TINY_CAM, keys, F, W, rgb_, gmc, grgb)
