"""torch.autograd.Function over the differentiable fusion entry points (vbh_diff_*).

The loss is L = sum_k F_tri(x_k)^2 after integrating n_frames depth maps into a fresh
volume; its inputs are the depth maps and a per-frame tangent perturbation xi = (rho; phi)
of the camera-to-world poses, applied on the left: T_f = Exp(xi_f) T_f.  The gradient
returned for xi is the left-perturbation gradient at the perturbed pose, which equals
dL/dxi at xi = 0 (the usual setting: xi is a zero tangent vector that requires grad).
All computation runs in libvbh; this module only marshals tensors.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from .binding import _check, _ptr, _stream, lib, vbh_params


def se3_exp(xi: np.ndarray) -> np.ndarray:
    """4x4 exponential of xi = (rho; phi) (Rodrigues rotation, V rho translation)."""
    rho, phi = np.asarray(xi[:3], np.float64), np.asarray(xi[3:], np.float64)
    th = float(np.linalg.norm(phi))
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    if th < 1e-6:
        A, B, Cc = 1 - th * th / 6, 0.5 - th * th / 24, 1 / 6 - th * th / 120
    else:
        A, B, Cc = np.sin(th) / th, (1 - np.cos(th)) / th ** 2, (th - np.sin(th)) / th ** 3
    R = np.eye(3) + A * K + B * K @ K
    V = np.eye(3) + B * K + Cc * K @ K
    T = np.eye(4)
    T[:3, :3], T[:3, 3] = R, V @ rho
    return T


class DiffFusion:
    """Owns a vbh_diff handle (a scene plus gradient buffers) on the current device."""

    def __init__(self, params: vbh_params, n_frames: int):
        self._L = lib()
        h = C.c_void_p()
        _check(lib().vbh_diff_create(C.byref(params), n_frames, C.byref(h)), "vbh_diff_create")
        self.h, self.params, self.n_frames = h, params, n_frames

    def close(self):
        # the library object is held by the instance: module globals may already be gone
        # when this runs at interpreter exit
        L = getattr(self, "_L", None)
        if getattr(self, "h", None) and L is not None:
            L.vbh_diff_destroy(self.h)
        self.h = None

    __del__ = close

    def _poses(self, poses):
        P = np.ascontiguousarray(np.asarray(poses, np.float64).reshape(self.n_frames, -1)[:, :12], np.float32)
        return P, P.ctypes.data_as(C.POINTER(C.c_float))

    def vbh_diff_forward(self, depth, poses, sample_frame, sample_pixel, with_samples=True):
        K = sample_frame.numel()
        P, pp = self._poses(poses)
        loss = torch.empty((), dtype=torch.float32, device=depth.device)
        fs = torch.empty(K, dtype=torch.float32, device=depth.device) if with_samples else None
        _check(lib().vbh_diff_forward(self.h, _ptr(depth, torch.float32, name="depth"), pp,
                                      _ptr(sample_frame, torch.int32, K), _ptr(sample_pixel, torch.int32, K), K,
                                      _ptr(fs), _ptr(loss), _stream()), "vbh_diff_forward")
        return loss, fs

    def vbh_diff_backward(self, depth, poses, sample_frame, sample_pixel, grad_loss):
        K = sample_frame.numel()
        P, pp = self._poses(poses)
        gD = torch.empty_like(depth)
        gxi = torch.empty((self.n_frames, 6), dtype=torch.float32, device=depth.device)
        gl = grad_loss.reshape(()).to(torch.float32).contiguous()
        _check(lib().vbh_diff_backward(self.h, _ptr(depth, torch.float32, name="depth"), pp,
                                       _ptr(sample_frame, torch.int32, K), _ptr(sample_pixel, torch.int32, K), K,
                                       _ptr(gl), _ptr(gD), _ptr(gxi), _stream()), "vbh_diff_backward")
        return gD, gxi


class TSDFSampleLoss(torch.autograd.Function):
    """loss = TSDFSampleLoss.apply(depth [F,H,W], xi [F,6], engine, poses [F,3,4],
    sample_frame [K] int32, sample_pixel [K] int32)."""

    @staticmethod
    def forward(ctx, depth, xi, engine: DiffFusion, poses, sample_frame, sample_pixel):
        xin = xi.detach().double().cpu().numpy()
        P0 = np.asarray(poses, np.float64).reshape(-1, 3, 4)
        Pf = np.stack([(se3_exp(xin[f]) @ np.vstack([P0[f], [0, 0, 0, 1]]))[:3] for f in range(P0.shape[0])])
        d = depth.detach().contiguous()
        loss, _ = engine.vbh_diff_forward(d, Pf, sample_frame, sample_pixel, with_samples=False)
        ctx.engine, ctx.poses = engine, Pf
        ctx.save_for_backward(d, sample_frame, sample_pixel)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        d, sf, sp = ctx.saved_tensors
        gD, gxi = ctx.engine.vbh_diff_backward(d, ctx.poses, sf, sp, grad_loss)
        return gD, gxi, None, None, None, None
