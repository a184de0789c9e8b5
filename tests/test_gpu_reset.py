"""GPU parity of the scene reset (Sec. 4.1, quasi-static scenes) and of the selection of the
currently visible blocks, against the oracle: visible sets bit-exact (the same float32
decisions), the reset's touched and MC sets and log bit-exact, and the whole volume
after reset and further fusion within the bar of the scene tests."""
import dataclasses

import numpy as np
import torch

import pytest
from datagen import configs
from gpu_util import keyset, require_gpu, say, to_dev
from test_gpu_scene import compare_state, integrate_both, make_pair

pytestmark = pytest.mark.gpu
VOL = dataclasses.replace(configs.TINY_VOL, depth_min=0.3, depth_max=1.1)
CAM = configs.TINY_CAM


def test_visible_blocks_equal_oracle(orc):
    vbh = require_gpu()
    _, depth, rgb, poses = configs.tiny_inputs(24)
    G, O = make_pair(vbh, orc, VOL, CAM)
    integrate_both(G, O, depth, rgb, poses, range(8), check_frames=False)
    n_all = O.n_blocks()
    for f in (0, 3, 7, 12, 20, 23):
        got = G.vbh_scene_visible_blocks(poses[f])
        want = O.visible_blocks(poses[f])
        say(f"[visible] pose {f}: {got.shape[0]} of {n_all} blocks")
        assert got.shape[0] == want.shape[0] and keyset(got) == keyset(want)
    # an empty scene has no visible block
    E = vbh.Scene(vbh.make_params(VOL, CAM))
    assert E.vbh_scene_visible_blocks(poses[0]).shape[0] == 0


def test_reset_then_refuse_equals_oracle(orc):
    vbh = require_gpu()
    _, depth, rgb, poses = configs.tiny_inputs(16)
    G, O = make_pair(vbh, orc, VOL, CAM)
    integrate_both(G, O, depth, rgb, poses, range(6))
    vis = O.visible_blocks(poses[2])
    absent = np.array([[900, 900, 900], [-900, 5, 5]], np.int32)
    req = np.concatenate([vis, vis[:7], absent])[np.random.default_rng(3).permutation(vis.shape[0] + 9)]
    mark = O.log_length()
    G.vbh_scene_reset_blocks(to_dev(req), 7)
    rc, n_reset = O.reset_blocks(req, 7)
    assert rc == 0 and G.vbh_scene_status() == 0
    st = G.vbh_scene_stats()
    say(f"[reset] {n_reset} blocks reset, MC set {st['n_mc']}, log {st['log_length']}")
    assert st["n_touched"] == n_reset and st["n_new"] == 0
    assert keyset(G.vbh_scene_last_touched()) == keyset(O.last_touched())
    assert keyset(G.vbh_scene_last_mc()) == keyset(O.last_mc_updated())
    assert st["log_length"] == O.log_length() and st["n_blocks"] == O.n_blocks()
    keys, meta = G.vbh_updated_blocks_since(mark, 1 << 20)
    n = int(meta[0])
    assert keyset(keys[:n]) == keyset(O.updated_since(mark, 1 << 20)[0])
    # reset blocks carry no data and no MC voxels
    F, W, c, found = G.vbh_scene_read_blocks(to_dev(vis))
    assert bool(found.all()) and not W.any() and not c.any() and not F.any()
    mc, mrgb = G.vbh_stored_mc(to_dev(vis))
    assert not mc.any() and not mrgb.any()
    compare_state(G, O)
    # fusion continues on the reset region
    integrate_both(G, O, depth, rgb, poses, range(6, 12), first_id=8)
    compare_state(G, O)
    # an all-absent reset is an empty update; frame ids must still increase
    G.vbh_scene_reset_blocks(to_dev(absent), 20)
    O.reset_blocks(absent, 20)
    assert G.vbh_scene_stats()["n_mc"] == 0 and G.vbh_scene_status() == 0
    with pytest.raises(vbh.VbhError):
        G.vbh_scene_reset_blocks(to_dev(vis), 20)


def test_reset_everything_equals_fresh_volume():
    """Reset every block, fuse the same frames again: the voxels equal those of a fresh
    volume that fused them (blocks only in the reset volume stay unobserved)."""
    vbh = require_gpu()
    _, depth, rgb, poses = configs.tiny_inputs(8)
    A = vbh.Scene(vbh.make_params(VOL, CAM))
    B = vbh.Scene(vbh.make_params(VOL, CAM))
    for f in range(4):
        A.vbh_integrate_frame(depth[f].cuda(), rgb[f].cuda(), poses[f], f + 1)
        B.vbh_integrate_frame(depth[f].cuda(), rgb[f].cuda(), poses[f], f + 1)
    for f in range(4, 8):
        A.vbh_integrate_frame(depth[f].cuda(), rgb[f].cuda(), poses[f], f + 1)
    A.vbh_scene_reset_blocks(A.vbh_scene_export_blocks(), 9)
    for f in range(4):
        A.vbh_integrate_frame(depth[f].cuda(), rgb[f].cuda(), poses[f], 10 + f)
    assert A.vbh_scene_status() == 0 and B.vbh_scene_status() == 0
    kb = B.vbh_scene_export_blocks()
    Fa, Wa, Ca, fa = A.vbh_scene_read_blocks(kb)
    Fb, Wb, Cb, _ = B.vbh_scene_read_blocks(kb)
    assert bool(fa.all())
    assert torch.equal(Wa, Wb) and torch.equal(Ca, Cb) and torch.equal(Fa, Fb)
    ka = A.vbh_scene_export_blocks()
    extra = [k for k in ka.cpu().numpy().tolist() if tuple(k) not in keyset(kb)]
    if extra:
        assert not A.vbh_scene_read_blocks(to_dev(np.array(extra, np.int32)))[1].any()
    # the MC voxels of B's blocks agree once recomputed from identical voxels
    ma, ca = A.vbh_extract_mc_indices(kb)
    mb, cb = B.vbh_extract_mc_indices(kb)
    assert torch.equal(ma, mb) and torch.equal(ca, cb)


def test_reset_reaches_serving_clients():
    """A client that streamed the scene before a reset receives, with its next requests
    through the serving loop, exactly the reset's update set, and the reset blocks as
    MC blocks with no surface (Sec. 4.1 reset propagated to the clients, Sec. 4.2)."""
    vbh = require_gpu()
    _, depth, rgb, poses = configs.tiny_inputs(8)
    S = vbh.Scene(vbh.make_params(VOL, CAM))
    for f in range(8):
        S.vbh_integrate_frame(depth[f].cuda(), rgb[f].cuda(), poses[f], f + 1)
    nb = S.vbh_scene_stats()["n_blocks"]
    srv = vbh.Server(S, arena_bytes=128 << 20, max_inflight=8, n_streams=2, n_clients=2, max_batch=4)
    lim = nb + 16
    outs = [(torch.zeros((lim, 3), dtype=torch.int32, device="cuda"),
             torch.zeros((lim, 512), dtype=torch.int32, device="cuda"))]
    r0 = srv.vbh_server_run([0], [lim], [0.0], outs)
    assert r0["status"][0] == 0 and r0["count"][0] == nb  # the client holds the whole model
    vis = S.vbh_scene_visible_blocks(poses[3])
    S.vbh_scene_reset_blocks(vis, 9)
    assert S.vbh_scene_status() == 0
    upd = keyset(S.vbh_scene_last_mc())
    r1 = srv.vbh_server_run([0], [lim], [0.0], outs)
    k = int(r1["count"][0])
    got = outs[0][0][:k]
    say(f"[reset serve] {vis.shape[0]} reset, {len(upd)} republished, {k} delivered")
    assert r1["status"][0] == 0 and keyset(got) == upd and k == len(upd)
    reset = keyset(vis)
    is_reset = torch.tensor([tuple(x) in reset for x in got.cpu().numpy().tolist()], device="cuda")
    mcs = outs[0][1][:k]
    assert not mcs[is_reset].any()  # no surface left in the reset blocks
    if bool((~is_reset).any()):
        assert mcs[~is_reset].any()  # refreshed neighbours keep their surface
