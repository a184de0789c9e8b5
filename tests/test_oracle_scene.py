"""Pins of the oracle's allocation, integration, MC voxel encoding and update log against
closed forms, hand-derived special cases and set algebra."""
import json
import math
import os

import numpy as np
import pytest

from datagen import configs
from datagen.configs import Volume
from datagen.scenes import Camera

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))

CAM = Camera(8, 6, 4.0, 4.0, 3.5, 2.5)
VOL = Volume(slots=1 << 12, pool_blocks=1 << 12, voxel_size=0.01, trunc=0.04, depth_min=0.0,
             depth_max=float("inf"), log_capacity=1 << 16)
IDENT = np.hstack([np.eye(3), np.zeros((3, 1))])


def plane_frame(D, cam=CAM):
    return np.full((cam.height, cam.width), D, np.float32)


def pick_depth(vol=VOL, cam=CAM):
    """A plane depth whose band samples all stay >= 1e-4 (relative) from block edges."""
    f32 = np.float32
    for D in np.arange(0.2031, 0.6, 0.00173):
        D = float(f32(D))
        ok = True
        for s in range(9):
            lam = float(f32(f32(D) - f32(vol.trunc)) + f32(s) * f32(vol.voxel_size))
            for u in range(cam.width):
                for c in (lam * (u - cam.cx) / cam.fx, lam * (0 - cam.cy) / cam.fy, lam):
                    q = c / (8 * float(f32(vol.voxel_size)))
                    if abs(q - round(q)) < 1e-3:
                        ok = False
        if ok:
            return D
    raise AssertionError("no suitable depth")


# ------------------------------------------------------------------------ allocation

def test_allocation_plane_closed_form(orc):
    D = pick_depth()
    S = orc.Scene(VOL, CAM)
    assert S.integrate(plane_frame(D), None, IDENT, 1) == 0
    got = {tuple(k) for k in S.last_touched()}
    vs, mu, bs = float(np.float32(0.01)), float(np.float32(0.04)), 8 * float(np.float32(0.01))
    want = set()
    for v in range(CAM.height):
        for u in range(CAM.width):
            for s in range(9):
                lam = (D - mu) + s * vs
                x, y = lam * (u - CAM.cx) / CAM.fx, lam * (v - CAM.cy) / CAM.fy
                want.add((math.floor(x / bs), math.floor(y / bs), math.floor(lam / bs)))
    assert got == want
    # every touched block intersects the slab z in [D-mu, D+mu]
    for (_, _, bz) in got:
        assert bz * bs <= D + mu + 1e-6 and (bz + 1) * bs >= D - mu - 1e-6
    assert {tuple(k) for k in S.last_new()} == got


def test_allocation_skips_invalid_and_counts_new(orc):
    D = pick_depth()
    d = plane_frame(D)
    d[0, :] = 0.0
    d[1, 2] = np.nan
    S = orc.Scene(VOL, CAM)
    S.integrate(d, None, IDENT, 1)
    n1 = len(S.last_touched())
    S.integrate(plane_frame(D), None, IDENT, 2)
    # second frame touches a superset; only the extra blocks are new
    t2 = {tuple(k) for k in S.last_touched()}
    assert len(t2) >= n1
    assert len(S.last_new()) == len(t2) - n1
    assert S.n_blocks() == len(t2)


def test_allocation_depth_range_gate(orc):
    vol = Volume(**{**VOL.__dict__, "depth_min": 0.4, "depth_max": 4.0})
    S = orc.Scene(vol, CAM)
    S.integrate(plane_frame(0.3), None, IDENT, 1)
    assert len(S.last_touched()) == 0
    S.integrate(plane_frame(4.5), None, IDENT, 2)
    assert len(S.last_touched()) == 0


def test_pool_exhaustion_is_reported(orc):
    vol = Volume(**{**VOL.__dict__, "pool_blocks": 3})
    S = orc.Scene(vol, CAM)
    rc = S.integrate(plane_frame(pick_depth()), None, IDENT, 1)
    assert rc == -5 and S.error() == -5 and S.n_blocks() == 3


# ----------------------------------------------------------------------- integration

def voxel_centres(keys):
    loc = np.arange(512)
    l = np.stack([loc % 8, (loc // 8) % 8, loc // 64], -1)
    return keys[:, None, :].astype(np.int64) * 8 + l[None]


def projection64(g, vs):
    p = g * vs
    with np.errstate(divide="ignore", invalid="ignore"):
        u = CAM.fx * (p[..., 0] / p[..., 2]) + CAM.cx + 0.5
        v = CAM.fy * (p[..., 1] / p[..., 2]) + CAM.cy + 0.5
    safe = (np.abs(u - np.round(u)) > 1e-4) & (np.abs(v - np.round(v)) > 1e-4) & (p[..., 2] > 0)
    inside = (u >= 0) & (u < CAM.width) & (v >= 0) & (v < CAM.height)
    return safe, inside


def test_integration_plane_closed_form(orc):
    D = pick_depth()
    S = orc.Scene(VOL, CAM)
    S.integrate(plane_frame(D), None, IDENT, 1)
    keys = S.blocks()
    F, W, _, found = S.read(keys)
    assert found.all()
    vs, mu = float(np.float32(0.01)), float(np.float32(0.04))
    g = voxel_centres(keys)
    z = g[..., 2] * vs
    sdf = D - z
    safe, inside = projection64(g.astype(np.float64), vs)
    obs = inside & (sdf >= -mu)
    m = safe
    assert (W[m] == obs[m]).all()
    want = np.minimum(sdf, mu)
    assert np.abs(F[m & obs] - want[m & obs]).max() < 1e-12
    # the true clamped signed distance to the plane (fronto-parallel) within 1e-6 m
    assert np.abs(F[m & obs] - np.minimum(D - z, mu)[m & obs]).max() < 1e-6
    assert (F[~obs & m] == 0).all()


def test_integration_running_mean_and_weight(orc):
    D1 = pick_depth()
    D2 = D1 + 0.0113
    S = orc.Scene(VOL, CAM)
    S.integrate(plane_frame(D1), None, IDENT, 1)
    S.integrate(plane_frame(D2), None, IDENT, 2)
    keys = S.blocks()
    F, W, _, _ = S.read(keys)
    vs, mu = float(np.float32(0.01)), float(np.float32(0.04))
    g = voxel_centres(keys)
    z = g[..., 2] * vs
    safe, inside = projection64(g.astype(np.float64), vs)
    t1 = np.minimum(np.float32(D1) - z, mu)
    t2 = np.minimum(np.float32(D2) - z, mu)
    both = safe & inside & (t1 >= -mu) & (np.float32(D2) - z >= -mu)
    assert (W[both] == 2).all()
    assert np.abs(F[both] - (t1[both] + t2[both]) / 2).max() < 1e-12


def test_weight_saturates_at_255(orc):
    cam = Camera(2, 2, 2.0, 2.0, 0.5, 0.5)
    S = orc.Scene(VOL, cam)
    D = 0.2537
    for f in range(300):
        S.integrate(np.full((2, 2), D, np.float32), None, IDENT, f + 1)
    keys = S.blocks()
    F, W, _, _ = S.read(keys)
    assert W.max() == 255
    g = voxel_centres(keys)
    tsdf = np.minimum(np.float32(D) - g[..., 2] * float(np.float32(0.01)), float(np.float32(0.04)))
    sat = W == 255
    assert np.abs(F[sat] - tsdf[sat]).max() < 1e-9


def test_colour_running_mean_round_half_up(orc):
    cam = Camera(2, 2, 2.0, 2.0, 0.5, 0.5)
    S = orc.Scene(VOL, cam)
    D = np.full((2, 2), 0.2537, np.float32)
    obs = [10, 11, 13, 200]
    want = [10, 11, 12, 59]  # (0+10+0)/1, (10+11+1)/2, (2*11+13+1)/3, (3*12+200+2)/4
    for f, c in enumerate(obs):
        S.integrate(D, np.full((2, 2, 3), c, np.uint8), IDENT, f + 1)
        _, W, rgb, _ = S.read(S.blocks())
        sel = W == f + 1
        assert sel.any()
        assert (rgb[sel] == want[f]).all()


def test_frame_id_must_increase(orc):
    S = orc.Scene(VOL, CAM)
    assert S.integrate(plane_frame(0.3), None, IDENT, 5) == 0
    assert S.integrate(plane_frame(0.3), None, IDENT, 5) == -1
    assert S.integrate(plane_frame(0.3), None, IDENT, 0) == -1


# ------------------------------------------------------------------------ MC voxels

def grid_blocks(fn, n=2, W=1):
    """Blocks (0..n-1)^3 with F = fn(global voxel index float64 [...,3])."""
    keys = np.array([(x, y, z) for x in range(n) for y in range(n) for z in range(n)], np.int32)
    g = voxel_centres(keys).astype(np.float64)
    F = fn(g).astype(np.float32)
    Wt = np.full(F.shape, W, np.uint8)
    rgb = np.zeros(F.shape + (3,), np.uint8)
    rgb[..., 0] = 7
    rgb[..., 1] = 99
    rgb[..., 2] = 201
    return keys, F, Wt, rgb


def mc_of(orc, keys, F, W, rgb, query):
    S = orc.Scene(VOL, CAM)
    assert S.write(keys, F, W, rgb, 1) == 0
    return S.extract_mc(np.asarray(query, np.int32))


def test_mc_all_outside_all_inside(orc):
    mc, rgb = mc_of(orc, *grid_blocks(lambda g: np.full(g.shape[:-1], 0.5)), [[0, 0, 0]])
    assert (mc == 0).all() and (rgb == 0).all()
    mc, rgb = mc_of(orc, *grid_blocks(lambda g: np.full(g.shape[:-1], -0.5)), [[0, 0, 0]])
    assert (mc == 0).all() and (rgb == 0).all()  # 255 is cut off as well


def test_mc_single_negative_corner_each_bit(orc):
    g0 = np.array([3, 4, 5])
    keys, F, W, rgb = grid_blocks(lambda g: np.where((g == g0).all(-1), -0.25, 0.25))
    mc, col = mc_of(orc, keys, F, W, rgb, [[0, 0, 0]])
    # corner k of cell c is voxel c + o_k; o_k in the Lorensen-Cline numbering
    offs = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
    expect = np.zeros(512, np.uint8)
    for k, o in enumerate(offs):
        c = g0 - np.array(o)
        expect[c[0] + 8 * c[1] + 64 * c[2]] = 1 << k
    assert np.array_equal(mc[0], expect)
    nz = expect > 0
    assert (col[0][nz] == [7, 99, 201]).all() and (col[0][~nz] == 0).all()


def test_mc_axis_plane(orc):
    keys, F, W, rgb = grid_blocks(lambda g: g[..., 2] - 3.5)  # negative below z = 3.5
    mc, _ = mc_of(orc, keys, F, W, rgb, [[0, 0, 0]])
    loc = np.arange(512)
    z = loc // 64
    assert (mc[0][z == 3] == 0x0F).all() and (mc[0][z != 3] == 0).all()
    keys, F, W, rgb = grid_blocks(lambda g: 3.5 - g[..., 2])  # negative above
    mc, _ = mc_of(orc, keys, F, W, rgb, [[0, 0, 0]])
    assert (mc[0][z == 3] == 0xF0).all() and (mc[0][z != 3] == 0).all()


def test_mc_missing_block_and_unobserved(orc):
    keys, F, W, rgb = grid_blocks(lambda g: g[..., 2] - 3.5, n=1)  # block (0,0,0) alone
    mc, _ = mc_of(orc, keys, F, W, rgb, [[0, 0, 0]])
    loc = np.arange(512)
    lx, ly, lz = loc % 8, (loc // 8) % 8, loc // 64
    face = (lx == 7) | (ly == 7) | (lz == 7)
    assert (mc[0][face] == 0).all()
    assert (mc[0][(lz == 3) & ~face] == 0x0F).all()
    keys, F, W, rgb = grid_blocks(lambda g: g[..., 2] - 3.5)
    W[0, 2 + 8 * 2 + 64 * 3] = 0  # one unobserved voxel at (2,2,3)
    mc, _ = mc_of(orc, keys, F, W, rgb, [[0, 0, 0]])
    for c in [(2, 2, 3), (1, 2, 3), (2, 1, 3), (1, 1, 3), (2, 2, 2), (1, 2, 2), (2, 1, 2), (1, 1, 2)]:
        assert mc[0][c[0] + 8 * c[1] + 64 * c[2]] == 0


def test_mc_sphere_matches_sign_pattern(orc):
    c0, r = np.array([7.3, 8.1, 6.6]), 4.7
    keys, F, W, rgb = grid_blocks(lambda g: np.linalg.norm(g - c0, axis=-1) - r)
    mc, _ = mc_of(orc, keys, F, W, rgb, [[0, 0, 0]])
    offs = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
    for l in range(512):
        g = np.array([l % 8, (l // 8) % 8, l // 64])
        idx = sum(1 << k for k, o in enumerate(offs) if np.linalg.norm(g + o - c0) < r)
        assert mc[0][l] == (0 if idx in GOLD["mc_cutoff_indices"]["value"] else idx)


def test_mc_store_matches_fresh_extraction(orc):
    _, depth, rgb, poses = configs.tiny_inputs(4)
    S = orc.Scene(configs.TINY_VOL, configs.TINY_CAM)
    for f in range(4):
        S.integrate(depth[f].numpy(), rgb[f].numpy(), poses[f], f + 1)
    keys = S.blocks()
    a = S.stored_mc(keys)
    b = S.extract_mc(keys)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert (a[0] > 0).sum() > 1000


# ----------------------------------------------------------------------- update log

def test_update_set_seven_negative_neighbours(orc):
    n7 = GOLD["mc_update_negative_neighbours"]["value"]
    keys, F, W, rgb = grid_blocks(lambda g: g[..., 2] - 3.5)
    S = orc.Scene(VOL, CAM)
    S.write(keys, F, W, rgb, 1)
    assert len(S.last_mc_updated()) == 8
    # rewrite only block (1,1,1): it and its seven negative neighbours are refreshed
    sel = [i for i, k in enumerate(keys) if tuple(k) == (1, 1, 1)]
    S.write(keys[sel], F[sel], W[sel], rgb[sel], 2)
    assert len(S.last_mc_updated()) == 1 + n7
    # rewrite block (0,0,0): its negative neighbours do not exist
    sel = [i for i, k in enumerate(keys) if tuple(k) == (0, 0, 0)]
    S.write(keys[sel], F[sel], W[sel], rgb[sel], 3)
    assert {tuple(k) for k in S.last_mc_updated()} == {(0, 0, 0)}


def test_updated_since_sets_and_pages(orc):
    _, depth, rgb, poses = configs.tiny_inputs(6)
    S = orc.Scene(configs.TINY_VOL, configs.TINY_CAM)
    marks = []
    for f in range(6):
        marks.append(S.log_length())
        S.integrate(depth[f].numpy(), rgb[f].numpy(), poses[f], f + 1)
    allk = {tuple(k) for k in S.blocks()}
    got, nxt = S.updated_since(0, 1 << 30)
    assert len(got) == len(allk) and {tuple(k) for k in got} == allk
    assert nxt == S.log_length()
    # the last frame's update set is exactly what is live after its log mark
    got, _ = S.updated_since(marks[-1], 1 << 30)
    assert {tuple(k) for k in got} == {tuple(k) for k in S.last_mc_updated()}
    # paging: union of pages = everything, no duplicates
    cur, seen = 0, []
    while True:
        page, cur2 = S.updated_since(cur, 97)
        seen += [tuple(k) for k in page]
        if len(page) < 97:
            break
        assert cur2 > cur
        cur = cur2
    assert len(seen) == len(set(seen)) and set(seen) == allk


# ------------------------------------------------- rotated pose (catches R vs R^T, t sign)

ROT_CAM = Camera(12, 10, 9.0, 9.0, 5.5, 4.5)


def rotated_setup():
    from datagen.scenes import look_at
    pose = look_at([0.031, -0.047, 0.023], [1.0, 0.35, -0.2])  # camera-to-world
    a = 0.6137  # wall x = a
    R, t = pose[:, :3], pose[:, 3]
    depth = np.zeros((ROT_CAM.height, ROT_CAM.width), np.float64)
    for v in range(ROT_CAM.height):
        for u in range(ROT_CAM.width):
            rw = R @ np.array([(u - ROT_CAM.cx) / ROT_CAM.fx, (v - ROT_CAM.cy) / ROT_CAM.fy, 1.0])
            depth[v, u] = (a - t[0]) / rw[0]  # c / (n . r)
    return pose, depth.astype(np.float32)


def test_allocation_rotated_pose(orc):
    pose, depth = rotated_setup()
    S = orc.Scene(VOL, ROT_CAM)
    S.integrate(depth, None, pose, 1)
    got = {tuple(k) for k in S.last_touched()}
    P = pose.astype(np.float32).astype(np.float64)
    R, t = P[:, :3], P[:, 3]
    vs, mu = float(np.float32(0.01)), float(np.float32(0.04))
    bs = 8 * vs
    strict, loose = set(), set()
    for v in range(ROT_CAM.height):
        for u in range(ROT_CAM.width):
            d = float(depth[v, u])
            for s in range(9):
                lam = (d - mu) + s * vs
                pc = lam * np.array([(u - ROT_CAM.cx) / ROT_CAM.fx, (v - ROT_CAM.cy) / ROT_CAM.fy, 1.0])
                q = (R @ pc + t) / bs
                B = np.floor(q).astype(int)
                near = np.abs(q - np.round(q)) < 1e-4
                if not near.any():
                    strict.add(tuple(B))
                for dx in ([0, -1] if near[0] else [0]):
                    for dy in ([0, -1] if near[1] else [0]):
                        for dz in ([0, -1] if near[2] else [0]):
                            loose.add((B[0] + dx, B[1] + dy, B[2] + dz))
                            loose.add((B[0] - dx, B[1] - dy, B[2] - dz))
    assert len(strict) > 10
    assert strict <= got <= loose


def test_integration_rotated_pose_closed_form(orc):
    pose, depth = rotated_setup()
    S = orc.Scene(VOL, ROT_CAM)
    S.integrate(depth, None, pose, 1)
    keys = S.blocks()
    F, W, _, _ = S.read(keys)
    P = pose.astype(np.float32).astype(np.float64)
    R, t = P[:, :3], P[:, 3]
    vs, mu = float(np.float32(0.01)), float(np.float32(0.04))
    X = voxel_centres(keys).astype(np.float64) * vs
    Xc = (X - t) @ R  # world -> camera: R^T (X - t)
    with np.errstate(divide="ignore", invalid="ignore"):
        uf = ROT_CAM.fx * Xc[..., 0] / Xc[..., 2] + ROT_CAM.cx + 0.5
        vf = ROT_CAM.fy * Xc[..., 1] / Xc[..., 2] + ROT_CAM.cy + 0.5
    safe = (np.abs(uf - np.round(uf)) > 1e-3) & (np.abs(vf - np.round(vf)) > 1e-3) & (Xc[..., 2] > 0)
    inside = (uf >= 0) & (uf < ROT_CAM.width) & (vf >= 0) & (vf < ROT_CAM.height)
    ui = np.clip(np.floor(np.nan_to_num(uf)).astype(int), 0, ROT_CAM.width - 1)
    vi = np.clip(np.floor(np.nan_to_num(vf)).astype(int), 0, ROT_CAM.height - 1)
    sdf = depth[vi, ui].astype(np.float64) - Xc[..., 2]
    obs = safe & inside & (sdf >= -mu + 1e-6)
    unobs = safe & (~inside | (sdf < -mu - 1e-6))
    assert obs.sum() > 200
    assert (W[obs] == 1).all() and (W[unobs] == 0).all()
    assert np.abs(F[obs] - np.minimum(sdf, mu)[obs]).max() < 1e-6


def test_power_of_two_world_scaling_is_exact(orc):
    """Multiplying every length (voxel size, truncation, depths, translations) by 2^30
    commutes with float rounding, so the float32 decisions (block keys, pixels, depth and
    truncation tests) are unchanged and the float64 F scales exactly: same blocks, W,
    colour, MC voxels and update log, F times 2^30.  A decision that mixed a length with
    a pure number in float (say an offset added in metres) would break it."""
    S = 2.0 ** 30
    _, depth, rgb, poses = configs.tiny_inputs(3)
    vol = configs.TINY_VOL
    vol_s = Volume(**{**vol.__dict__, "voxel_size": vol.voxel_size * S, "trunc": vol.trunc * S})
    poses_s = poses.copy()
    poses_s[..., 3] *= S
    A, B = orc.Scene(vol, configs.TINY_CAM), orc.Scene(vol_s, configs.TINY_CAM)
    for f in range(3):
        assert A.integrate(depth[f].numpy(), rgb[f].numpy(), poses[f], f + 1) == 0
        assert B.integrate((depth[f] * S).numpy(), rgb[f].numpy(), poses_s[f], f + 1) == 0
        assert np.array_equal(np.sort(A.last_touched(), axis=0), np.sort(B.last_touched(), axis=0))
    ka, kb = A.blocks(), B.blocks()
    order = np.lexsort(ka.T[::-1])
    ka = ka[order]
    assert ka.shape == kb.shape and set(map(tuple, ka.tolist())) == set(map(tuple, kb.tolist()))
    Fa, Wa, ca, _ = A.read(ka)
    Fb, Wb, cb, _ = B.read(ka)
    assert np.array_equal(Wa, Wb) and np.array_equal(ca, cb)
    assert np.array_equal(Fa * S, Fb)
    ma, ra = A.stored_mc(ka)
    mb, rb = B.stored_mc(ka)
    assert np.array_equal(ma, mb) and np.array_equal(ra, rb)
    assert A.log_length() == B.log_length()
    la, lb = A.updated_since(0, 1 << 20), B.updated_since(0, 1 << 20)
    for x, y in zip(la, lb):
        assert np.array_equal(np.asarray(x), np.asarray(y))
