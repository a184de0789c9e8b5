"""Analytic scenes, an FP64 ray caster, Kinect-style depth noise and camera paths.

The paper measures on recorded RGB-D sequences that are not available here; these
generators stand in for them with the same shapes (640x480 or 320x240 depth in metres,
RGB8, 0.4-4 m range, axial noise growing with depth, dropout pixels).

Conventions (world metres, z up; camera OpenCV x right / y down / z forward; pose is
camera-to-world R|t with R columns = camera axes in world coordinates; depth is the
camera-z of the first hit, 0 = invalid).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


@dataclass
class Scene:
    """Union of solids inside a room.

    room:    (lo[3], hi[3]) axis-aligned interior the cameras live in
    boxes:   list of (lo[3], hi[3]) solid axis-aligned boxes
    spheres: list of (centre[3], radius)
    albedo:  per primitive RGB in [0,1]; index 0 = room, then boxes, then spheres
    """
    room: tuple
    boxes: list = field(default_factory=list)
    spheres: list = field(default_factory=list)
    albedo: list = field(default_factory=list)
    checker: float = 0.1


def _offset(vs: float) -> np.ndarray:
    # Shift all geometry off the voxel lattice so no wall lies within 0.1 voxel of a
    # lattice plane (avoids exact-zero TSDF ties at sign tests).
    return np.array([0.37, 0.41, 0.43]) * vs


def box_room_scene(seed: int = 1805, vs: float = 0.01) -> Scene:
    """2x2x2 m box room centred at the origin with three seed-placed spheres
    (radius U(0.2,0.4), centre uniform in a disk of radius 0.35 and |z|<=0.5, kept at
    least r+0.15 m from the radius-0.8 camera circle)."""
    rng = np.random.default_rng(seed)
    off = _offset(vs)
    room = (np.array([-1.0, -1.0, -1.0]) + off, np.array([1.0, 1.0, 1.0]) + off)
    spheres = []
    while len(spheres) < 3:
        r = rng.uniform(0.2, 0.4)
        a = rng.uniform(0, 2 * math.pi)
        rad = 0.35 * math.sqrt(rng.uniform(0, 1))
        c = np.array([rad * math.cos(a), rad * math.sin(a), rng.uniform(-0.5, 0.5)])
        dist_circle = math.hypot(math.hypot(c[0], c[1]) - 0.8, c[2])
        if dist_circle >= r + 0.15:
            spheres.append((c + off, r))
    albedo = [rng.uniform(0.3, 1.0, 3) for _ in range(1 + len(spheres))]
    return Scene(room=room, boxes=[], spheres=spheres, albedo=albedo)


def room_of_boxes_scene(seed: int = 5203, vs: float = 0.005, size=(10.0, 10.0, 3.0),
                        n_boxes: int = 20, n_spheres: int = 10) -> Scene:
    """Room [-sx/2,sx/2]x[-sy/2,sy/2]x[0,sz] with axis-aligned boxes (sides
    U(0.2,1.5) m) resting on the floor and floating spheres (r U(0.15,0.6) m)."""
    rng = np.random.default_rng(seed)
    off = _offset(vs)
    sx, sy, sz = size
    lo = np.array([-sx / 2, -sy / 2, 0.0])
    hi = np.array([sx / 2, sy / 2, sz])
    boxes, spheres = [], []
    for _ in range(n_boxes):
        s = rng.uniform(0.2, 1.5, 3)
        cx = rng.uniform(lo[0] + s[0] / 2, hi[0] - s[0] / 2)
        cy = rng.uniform(lo[1] + s[1] / 2, hi[1] - s[1] / 2)
        blo = np.array([cx - s[0] / 2, cy - s[1] / 2, 0.0])
        boxes.append((blo + off, blo + s + off))
    for _ in range(n_spheres):
        r = rng.uniform(0.15, 0.6)
        c = np.array([rng.uniform(lo[0] + r, hi[0] - r), rng.uniform(lo[1] + r, hi[1] - r),
                      rng.uniform(r, sz - r)])
        spheres.append((c + off, r))
    albedo = [rng.uniform(0.3, 1.0, 3) for _ in range(1 + n_boxes + n_spheres)]
    return Scene(room=(lo + off, hi + off), boxes=boxes, spheres=spheres, albedo=albedo)


def look_at(eye, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Camera-to-world 3x4 pose (float64) looking from eye to target."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    pose = np.zeros((3, 4))
    pose[:, 0], pose[:, 1], pose[:, 2], pose[:, 3] = r, d, f, eye
    return pose


def pose_from_yaw_pitch(eye, yaw: float, pitch: float) -> np.ndarray:
    f = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw),
                  math.sin(pitch)])
    return look_at(eye, np.asarray(eye) + f)


# ----------------------------------------------------------------------------- SDF

def _sd_box(p: torch.Tensor, lo, hi) -> torch.Tensor:
    lo = torch.as_tensor(lo, dtype=p.dtype, device=p.device)
    hi = torch.as_tensor(hi, dtype=p.dtype, device=p.device)
    c, h = (lo + hi) / 2, (hi - lo) / 2
    q = (p - c).abs() - h
    outside = q.clamp(min=0).norm(dim=-1)
    inside = q.max(dim=-1).values.clamp(max=0)
    return outside + inside


def scene_sdf(scene: Scene, p: torch.Tensor) -> torch.Tensor:
    """Signed distance to the scene surface, positive in free space (FP64 if p is)."""
    d = -_sd_box(p, *scene.room)
    for lo, hi in scene.boxes:
        d = torch.minimum(d, _sd_box(p, lo, hi))
    for c, r in scene.spheres:
        cc = torch.as_tensor(c, dtype=p.dtype, device=p.device)
        d = torch.minimum(d, (p - cc).norm(dim=-1) - r)
    return d


# ------------------------------------------------------------------------ ray cast

def _rays(cam: Camera, pose: np.ndarray, device, dtype=torch.float64):
    v, u = torch.meshgrid(torch.arange(cam.height, device=device, dtype=dtype),
                          torch.arange(cam.width, device=device, dtype=dtype), indexing="ij")
    dc = torch.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, torch.ones_like(u)], -1)
    R = torch.as_tensor(pose[:, :3], dtype=dtype, device=device)
    o = torch.as_tensor(pose[:, 3], dtype=dtype, device=device)
    d = dc @ R.T  # world direction whose camera-z component is 1
    return o, d


def raycast(scene: Scene, cam: Camera, pose: np.ndarray, device="cpu"):
    """FP64 ray cast; returns (depth float64 [H,W] as camera-z, primitive id int64 [H,W],
    world hit points float64 [H,W,3])."""
    o, d = _rays(cam, pose, device)
    inf = torch.tensor(float("inf"), dtype=torch.float64, device=device)
    # room interior: exit distance along each axis
    lo = torch.as_tensor(scene.room[0], dtype=torch.float64, device=device)
    hi = torch.as_tensor(scene.room[1], dtype=torch.float64, device=device)
    bound = torch.where(d > 0, hi, lo)
    with torch.no_grad():
        tw = torch.where(d != 0, (bound - o) / d, inf)
    t = tw.min(dim=-1).values
    pid = torch.zeros(t.shape, dtype=torch.int64, device=device)
    k = 1
    for blo, bhi in scene.boxes:
        blo = torch.as_tensor(blo, dtype=torch.float64, device=device)
        bhi = torch.as_tensor(bhi, dtype=torch.float64, device=device)
        t1 = (blo - o) / d
        t2 = (bhi - o) / d
        tn = torch.minimum(t1, t2).max(dim=-1).values
        tf = torch.maximum(t1, t2).min(dim=-1).values
        hit = (tn <= tf) & (tn > 0) & (tn < t)
        t = torch.where(hit, tn, t)
        pid = torch.where(hit, torch.full_like(pid, k), pid)
        k += 1
    for c, r in scene.spheres:
        cc = torch.as_tensor(c, dtype=torch.float64, device=device)
        oc = o - cc
        a = (d * d).sum(-1)
        b = 2 * (d * oc).sum(-1)
        c0 = (oc * oc).sum() - r * r
        disc = b * b - 4 * a * c0
        ts = (-b - disc.clamp(min=0).sqrt()) / (2 * a)
        hit = (disc >= 0) & (ts > 0) & (ts < t)
        t = torch.where(hit, ts, t)
        pid = torch.where(hit, torch.full_like(pid, k), pid)
        k += 1
    t = torch.where(torch.isfinite(t), t, torch.zeros_like(t))
    pts = o + t[..., None] * d
    return t, pid, pts


def shade(scene: Scene, pid: torch.Tensor, pts: torch.Tensor) -> torch.Tensor:
    """RGB8 albedo render: per-primitive albedo times a world-space checker."""
    alb = torch.as_tensor(np.stack(scene.albedo), dtype=torch.float64, device=pts.device)
    cell = torch.floor(pts / scene.checker).sum(-1).remainder(2)
    fac = torch.where(cell > 0, 1.0, 0.6)
    rgb = alb[pid] * fac[..., None] * 255.0
    return rgb.round().clamp(0, 255).to(torch.uint8)


def kinect_noise(z: torch.Tensor, frame_seed: int, zmin=0.4, zmax=4.0, dropout=0.02,
                 noise=True) -> torch.Tensor:
    """Axial noise sigma = 0.0012 + 0.0019 (z-0.4)^2 (Nguyen, Izadi, Lovell 2012),
    out-of-range depth set to 0, then Bernoulli dropout.  FP64 in, float32 out."""
    rng = np.random.default_rng(frame_seed)
    n = z.numel()
    g = torch.as_tensor(rng.standard_normal(n), device=z.device).view(z.shape)
    drop = torch.as_tensor(rng.random(n) < dropout, device=z.device).view(z.shape)
    valid = (z >= zmin) & (z <= zmax)
    sigma = 0.0012 + 0.0019 * (z - 0.4) ** 2
    zn = z + sigma * g if noise else z
    zn = torch.where(valid & ~drop, zn, torch.zeros_like(zn))
    return zn.to(torch.float32)


def render_frames(scene: Scene, cam: Camera, poses, device="cpu", noise_seed=None,
                  zmin=0.4, zmax=4.0, dropout=0.02, first_frame=0):
    """Render float32 depth [F,H,W] and RGB8 [F,H,W,3].  With noise_seed=None the depth
    is the noise-free FP64 cast rounded to float32; otherwise Kinect noise with seed
    noise_seed + frame index is applied."""
    depths, rgbs = [], []
    for i, pose in enumerate(poses):
        t, pid, pts = raycast(scene, cam, pose, device)
        if noise_seed is None:
            depths.append(t.to(torch.float32))
        else:
            depths.append(kinect_noise(t, noise_seed + first_frame + i, zmin, zmax, dropout))
        rgbs.append(shade(scene, pid, pts))
    return torch.stack(depths), torch.stack(rgbs)


def trajectory_c3(scene: Scene, n_frames: int, seed: int = 5203, fps: float = 30.0,
                  speed: float = 0.4, max_turn: float = 0.5, clearance: float = 0.5):
    """Smooth random walk inside the room: constant 0.4 m/s speed, heading driven by
    low-pass filtered Gaussian increments, height 1.2-1.8 m, yaw/pitch rates bounded
    by 0.5 rad/s, keeping >= 0.5 m from all geometry.  Returns [n,3,4] float64 poses."""
    rng = np.random.default_rng(seed + 7)
    step = speed / fps
    dmax = max_turn / fps

    def free(p):
        return scene_sdf(scene, torch.tensor(p, dtype=torch.float64)).item() >= clearance

    while True:
        p = np.array([rng.uniform(scene.room[0][0], scene.room[1][0]),
                      rng.uniform(scene.room[0][1], scene.room[1][1]), 1.5])
        if free(p):
            break
    heading = rng.uniform(0, 2 * math.pi)
    omega = 0.0
    yaw, pitch, pitch_rate = heading, -0.15, 0.0
    phase = rng.uniform(0, 2 * math.pi)
    poses = []
    for f in range(n_frames):
        z = 1.5 + 0.3 * math.sin(2 * math.pi * f / (fps * 20.0) + phase)
        poses.append(pose_from_yaw_pitch([p[0], p[1], z], yaw, pitch))
        omega = 0.9 * omega + 0.1 * rng.normal(0, dmax)
        omega = max(-dmax, min(dmax, omega))
        for attempt in range(64):
            h = heading + omega + (0 if attempt == 0 else rng.uniform(-math.pi, math.pi))
            q = p + step * np.array([math.cos(h), math.sin(h), 0.0])
            zq = 1.5 + 0.3 * math.sin(2 * math.pi * (f + 1) / (fps * 20.0) + phase)
            if free([q[0], q[1], zq]):
                heading, p = h, q
                break
        # yaw follows the heading with a bounded rate; pitch wanders in [-0.4, 0.1]
        dy = (heading - yaw + math.pi) % (2 * math.pi) - math.pi
        yaw += max(-dmax, min(dmax, dy))
        pitch_rate = 0.9 * pitch_rate + 0.1 * rng.normal(0, dmax)
        pitch = max(-0.4, min(0.1, pitch + max(-dmax, min(dmax, pitch_rate))))
    return np.stack(poses)
