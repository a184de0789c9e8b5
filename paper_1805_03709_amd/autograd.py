"""torch.autograd.Function over the differentiable fusion entry points (vbh_diff_*).

The loss is L = sum_k F_tri(x_k)^2 after integrating n_frames depth maps into a fresh
volume; its inputs are the depth maps and a per-frame tangent vector xi = (rho; phi) that
sets the camera-to-world poses T_f = Exp(xi_f) T0_f from base poses T0.  libvbh composes
the poses and returns dL/dxi (the left-perturbation gradient mapped through the SE(3)
left Jacobian of xi), so the gradient is exact at any xi, not only at xi = 0.  This
module only marshals tensors.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from .binding import _check, _ptr, _stream, lib, vbh_params


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

    def _xi(self, xi):
        return None if xi is None else _ptr(xi, torch.float32, 6 * self.n_frames, name="xi")

    def vbh_diff_forward(self, depth, poses, sample_frame, sample_pixel, xi=None, with_samples=True):
        K = sample_frame.numel()
        P, pp = self._poses(poses)
        loss = torch.empty((), dtype=torch.float32, device=depth.device)
        fs = torch.empty(K, dtype=torch.float32, device=depth.device) if with_samples else None
        _check(lib().vbh_diff_forward(self.h, _ptr(depth, torch.float32, name="depth"), pp, self._xi(xi),
                                      _ptr(sample_frame, torch.int32, K), _ptr(sample_pixel, torch.int32, K), K,
                                      _ptr(fs), _ptr(loss), _stream()), "vbh_diff_forward")
        return loss, fs

    def vbh_diff_backward(self, depth, poses, sample_frame, sample_pixel, grad_loss, xi=None):
        K = sample_frame.numel()
        P, pp = self._poses(poses)
        gD = torch.empty_like(depth)
        gxi = torch.empty((self.n_frames, 6), dtype=torch.float32, device=depth.device)
        gl = grad_loss.reshape(()).to(torch.float32).contiguous()
        _check(lib().vbh_diff_backward(self.h, _ptr(depth, torch.float32, name="depth"), pp, self._xi(xi),
                                       _ptr(sample_frame, torch.int32, K), _ptr(sample_pixel, torch.int32, K), K,
                                       _ptr(gl), _ptr(gD), _ptr(gxi), _stream()), "vbh_diff_backward")
        return gD, gxi


class TSDFSampleLoss(torch.autograd.Function):
    """loss = TSDFSampleLoss.apply(depth [F,H,W], xi [F,6], engine, poses [F,3,4],
    sample_frame [K] int32, sample_pixel [K] int32), with poses the base poses T0."""

    @staticmethod
    def forward(ctx, depth, xi, engine: DiffFusion, poses, sample_frame, sample_pixel):
        d = depth.detach().contiguous()
        x = xi.detach().to(torch.float32).contiguous()
        loss, _ = engine.vbh_diff_forward(d, poses, sample_frame, sample_pixel, xi=x, with_samples=False)
        ctx.engine, ctx.poses = engine, poses
        ctx.save_for_backward(d, x, sample_frame, sample_pixel)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        d, x, sf, sp = ctx.saved_tensors
        gD, gxi = ctx.engine.vbh_diff_backward(d, ctx.poses, sf, sp, grad_loss, xi=x)
        return gD, gxi.to(x.dtype), None, None, None, None
