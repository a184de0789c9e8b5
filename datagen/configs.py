"""The five workloads (sizes, seeds, volume parameters) and their input builders.

tiny   : 32 noise-free 320x240 frames around a 2 m box room with 3 spheres, 1 cm voxels
hash   : 2^24 keys (2^23 unique, each twice) in [-1024,1024)^3, 2^25 slots, 16 mixed
         1M-op batches
full   : 2000 noisy 640x480 frames along a random walk in a 10x10x3 m room of boxes and
         spheres, 5 mm voxels, 2 cm truncation, 2^22 slots
diff   : frames 500-515 of `full` into a 2 cm volume, 8 cm truncation, 100k samples
serve  : ~2M blocks analytically filled, 64 clients, Poisson requests
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from .scenes import (Camera, box_room_scene, look_at, render_frames, room_of_boxes_scene,
                     scene_sdf, trajectory_c3)


@dataclass
class Volume:
    slots: int
    pool_blocks: int
    voxel_size: float
    trunc: float
    depth_min: float
    depth_max: float
    log_capacity: int


TINY_CAM = Camera(320, 240, 285.0, 285.0, 159.5, 119.5)
FULL_CAM = Camera(640, 480, 525.0, 525.0, 319.5, 239.5)

TINY_VOL = Volume(slots=1 << 16, pool_blocks=1 << 15, voxel_size=0.01, trunc=0.04,
                  depth_min=0.0, depth_max=float("inf"), log_capacity=1 << 20)
FULL_VOL = Volume(slots=1 << 22, pool_blocks=1 << 21, voxel_size=0.005, trunc=0.02,
                  depth_min=0.4, depth_max=4.0, log_capacity=1 << 26)
SERVE_VOL = Volume(slots=1 << 23, pool_blocks=1 << 22, voxel_size=0.005, trunc=0.02,
                   depth_min=0.4, depth_max=4.0, log_capacity=1 << 26)
DIFF_VOL = Volume(slots=1 << 20, pool_blocks=1 << 16, voxel_size=0.02, trunc=0.08,
                  depth_min=0.4, depth_max=4.0, log_capacity=1 << 20)


def tiny_poses(n: int = 32) -> np.ndarray:
    return np.stack([look_at([0.8 * math.cos(2 * math.pi * k / n), 0.8 * math.sin(2 * math.pi * k / n), 0.0],
                             [0.0, 0.0, 0.0]) for k in range(n)])


def tiny_inputs(n_frames: int = 32, device="cpu", cam: Camera = TINY_CAM, seed: int = 1805):
    """Noise-free float32 depth [F,H,W], RGB8 [F,H,W,3] and float64 poses [F,3,4]."""
    scene = box_room_scene(seed, TINY_VOL.voxel_size)
    poses = tiny_poses(32)[:n_frames]
    depth, rgb = render_frames(scene, cam, poses, device=device)
    return scene, depth, rgb, poses


def full_scene(seed: int = 5203):
    return room_of_boxes_scene(seed, FULL_VOL.voxel_size)


def full_inputs(frames, device="cpu", seed: int = 5203, cam: Camera = FULL_CAM):
    """Noisy Kinect-shaped frames of the full workload; `frames` is a range/list of
    indices into the 2000-frame trajectory."""
    frames = list(frames)
    scene = full_scene(seed)
    traj = trajectory_c3(scene, max(frames) + 1, seed)
    poses = traj[frames]
    depths, rgbs = [], []
    for f, pose in zip(frames, poses):
        d, c = render_frames(scene, cam, [pose], device=device, noise_seed=seed, first_frame=f)
        depths.append(d[0])
        rgbs.append(c[0])
    return scene, torch.stack(depths), torch.stack(rgbs), poses


def diff_inputs(device="cpu", n_samples: int = 100_000, seed: int = 4242, first: int = 500,
                n_frames: int = 16, cam: Camera = FULL_CAM):
    """16 consecutive frames of the full trajectory and K pixel samples drawn uniformly
    without replacement from their valid pixels (depth inside the volume's range): returns (scene, depth, rgb, poses,
    sample_frame int32 [K], sample_pixel int32 [K] = v*W+u)."""
    scene, depth, rgb, poses = full_inputs(range(first, first + n_frames), device=device)
    valid = ((depth >= DIFF_VOL.depth_min) & (depth <= DIFF_VOL.depth_max)).reshape(-1).cpu().numpy()
    idx = np.flatnonzero(valid)
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(idx, size=min(n_samples, idx.size), replace=False))
    hw = cam.width * cam.height
    return scene, depth, rgb, poses, (pick // hw).astype(np.int32), (pick % hw).astype(np.int32)


def serve_scene(seed: int = 6464):
    """20x20x3 m room of 80 boxes and 40 spheres: about 2M blocks at 5 mm voxels."""
    return room_of_boxes_scene(seed, SERVE_VOL.voxel_size, size=(20.0, 20.0, 3.0), n_boxes=80, n_spheres=40)


def serve_frames(n_unique: int, device="cpu", seed: int = 6464, cam: Camera = FULL_CAM):
    """n_unique noisy 640x480 frames (depth, RGB, poses) along a random walk in the serving
    scene; callers cycle through them to fuse frames at 30 Hz."""
    scene = serve_scene(seed)
    traj = trajectory_c3(scene, n_unique, seed)
    depth = torch.empty((n_unique, cam.height, cam.width), dtype=torch.float32, device=device)
    rgb = torch.empty((n_unique, cam.height, cam.width, 3), dtype=torch.uint8, device=device)
    for f in range(n_unique):
        d, c = render_frames(scene, cam, [traj[f]], device=device, noise_seed=seed, first_frame=f)
        depth[f], rgb[f] = d[0], c[0]
    return depth, rgb, traj


def analytic_blocks(scene, voxel_size: float, trunc: float, device="cpu", seed: int = 6464,
                    chunk: int = 1 << 16):
    """Every 8^3 block whose centre lies within trunc + half the block diagonal of the
    surface, with F = clamp(exact SDF at the voxel lattice point, -trunc, trunc),
    W ~ U{1..255} and a grey checker colour.  Returns int32 keys [n,3], float32 F [n,512],
    uint8 W [n,512], uint8 RGB [n,512,3]."""
    bs = 8 * voxel_size
    lo = np.floor(scene.room[0] / bs).astype(np.int64) - 1
    hi = np.floor(scene.room[1] / bs).astype(np.int64) + 1
    ax = [torch.arange(lo[i], hi[i] + 1, device=device, dtype=torch.int64) for i in range(3)]
    keys = []
    rad = trunc + bs * math.sqrt(3) / 2
    for x in ax[0].split(16):
        g = torch.stack(torch.meshgrid(x, ax[1], ax[2], indexing="ij"), -1).reshape(-1, 3)
        c = (g.to(torch.float64) + 0.5) * bs
        keep = scene_sdf(scene, c).abs() <= rad
        keys.append(g[keep])
    keys = torch.cat(keys).to(torch.int32)
    loc = torch.arange(512, device=device)
    lvox = torch.stack([loc % 8, (loc // 8) % 8, loc // 64], -1)
    rng = np.random.default_rng(seed)
    F = torch.empty(keys.shape[0], 512, dtype=torch.float32, device=device)
    for s in range(0, keys.shape[0], chunk):
        kk = keys[s:s + chunk].to(torch.int64)
        gv = kk[:, None, :] * 8 + lvox[None]
        p = gv.to(torch.float64) * voxel_size
        F[s:s + chunk] = scene_sdf(scene, p).clamp(-trunc, trunc).to(torch.float32)
    W = torch.as_tensor(rng.integers(1, 256, size=(keys.shape[0], 512), dtype=np.uint8), device=device)
    rgb = torch.empty(keys.shape[0], 512, 3, dtype=torch.uint8, device=device)
    for s in range(0, keys.shape[0], chunk):
        gv = keys[s:s + chunk].to(torch.int64)[:, None, :] * 8 + lvox[None]
        grey = torch.where(gv.sum(-1).remainder(2) > 0, 200, 90).to(torch.uint8)
        rgb[s:s + chunk] = torch.stack([grey, grey, (grey // 2 + 60).to(torch.uint8)], -1)
    return keys, F, W, rgb
