"""ctypes binding of libvbh.so (include/vbh.h).

Argument marshalling only: every step of the hot path runs in the library's HIP kernels.
Device buffers are torch tensors on a HIP device (PyTorch supplies memory and streams);
work is enqueued on torch's current stream.  torch is imported before the library is
loaded so both share one HIP runtime.  If the library is not built this module raises -
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

import torch

from .build import LIB

VBH_OK, VBH_EINVAL, VBH_ENOMEM, VBH_EHIP = 0, -1, -2, -3
VBH_EFULL_TABLE, VBH_EFULL_POOL, VBH_EFULL_LOG, VBH_ESPIN = -4, -5, -6, -7
VBH_ABSENT = -(1 << 31)
VBH_OP_INSERT, VBH_OP_FIND, VBH_OP_ERASE = 0, 1, 2
VBH_HASH_SPATIAL, VBH_HASH_MIX64 = 0, 1

_lib = None


class VbhError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = _load().vbh_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


class vbh_params(C.Structure):
    _fields_ = [("slots", C.c_uint64), ("pool_blocks", C.c_int64), ("log_capacity", C.c_int64),
                ("voxel_size", C.c_float), ("trunc", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("depth_min", C.c_float), ("depth_max", C.c_float), ("hash_kind", C.c_int32)]


class vbh_stats(C.Structure):
    _fields_ = [("n_touched", C.c_int64), ("n_new", C.c_int64), ("n_mc", C.c_int64),
                ("n_voxel_updates", C.c_int64), ("n_blocks", C.c_int64), ("log_length", C.c_uint64),
                ("last_frame", C.c_uint32), ("error", C.c_int32), ("total_touched", C.c_int64),
                ("total_mc", C.c_int64), ("total_voxel_updates", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vbh_server_config(C.Structure):
    _fields_ = [("arena_bytes", C.c_int64), ("max_inflight", C.c_int32), ("n_streams", C.c_int32),
                ("n_clients", C.c_int32), ("max_batch", C.c_int32), ("mode", C.c_int32), ("workgroups", C.c_int32)]


class vbh_request(C.Structure):
    _fields_ = [("client", C.c_int32), ("reserved", C.c_int32), ("limit", C.c_int64), ("arrival_s", C.c_double),
                ("d_keys_out", C.c_void_p), ("d_mc_out", C.c_void_p)]


class vbh_request_result(C.Structure):
    _fields_ = [("arrival_s", C.c_double), ("admit_s", C.c_double), ("done_s", C.c_double),
                ("count", C.c_int64), ("cursor_in", C.c_uint64), ("cursor_out", C.c_uint64),
                ("version", C.c_uint32), ("status", C.c_int32)]


class vbh_frame_feed(C.Structure):
    _fields_ = [("d_depth", C.c_void_p), ("d_rgb", C.c_void_p), ("pose_c2w", C.c_float * 12),
                ("time_s", C.c_double), ("frame_id", C.c_uint32), ("reserved", C.c_uint32)]


_V, _I64, _U64, _I32, _P = C.c_void_p, C.c_int64, C.c_uint64, C.c_int32, C.c_void_p
SIGNATURES = {
    "vbh_strerror": ([C.c_int], C.c_char_p),
    "vbh_version": ([], C.c_int),
    "vbh_map_create": ([_U64, _I32, C.POINTER(_V)], C.c_int),
    "vbh_map_create_chained": ([_U64, _U64, _I32, C.POINTER(_V)], C.c_int),
    "vbh_map_destroy": ([_V], None),
    "vbh_insert": ([_V, _P, _P, _I64, _P, _V], C.c_int),
    "vbh_find": ([_V, _P, _I64, _P, _V], C.c_int),
    "vbh_erase": ([_V, _P, _I64, _P, _V], C.c_int),
    "vbh_apply": ([_V, _P, _P, _P, _I64, _P, _V], C.c_int),
    "vbh_map_size": ([_V, C.POINTER(_I64), C.POINTER(_I64), _V], C.c_int),
    "vbh_map_export": ([_V, _P, _P, _I64, C.POINTER(_I64), _V], C.c_int),
    "vbh_map_rebuild": ([_V, _V], C.c_int),
    "vbh_map_clear": ([_V, _V], C.c_int),
    "vbh_map_status": ([_V, _V], C.c_int),
    "vbh_size": ([_V, C.POINTER(_I64), _V], C.c_int),
    "vbh_status": ([_V, _V], C.c_int),
    "vbh_extract_mc_all": ([_V, _P, _I64, _P, _P, C.POINTER(_I64), _V], C.c_int),
    "vbh_scene_create": ([C.POINTER(vbh_params), C.POINTER(_V)], C.c_int),
    "vbh_scene_destroy": ([_V], None),
    "vbh_integrate_frame": ([_V, _P, _P, C.POINTER(C.c_float), C.c_uint32, _V], C.c_int),
    "vbh_integrate_blocks": ([_V, _P, _I64, _P, _P, C.POINTER(C.c_float), C.c_uint32, _V], C.c_int),
    "vbh_integrate_frames": ([_V, _P, _P, C.POINTER(C.c_float), C.c_uint32, _I64, _V], C.c_int),
    "vbh_integrate_frames_host": ([_V, _P, _P, C.POINTER(C.c_float), C.c_uint32, _I64, _V], C.c_int),
    "vbh_extract_mc_indices": ([_V, _P, _I64, _P, _P, _V], C.c_int),
    "vbh_stored_mc": ([_V, _P, _I64, _P, _P, _V], C.c_int),
    "vbh_updated_blocks_since": ([_V, _U64, _I64, _P, _P, _P, _V], C.c_int),
    "vbh_scene_status": ([_V, _V], C.c_int),
    "vbh_scene_stats": ([_V, C.POINTER(vbh_stats), _V], C.c_int),
    "vbh_scene_export_blocks": ([_V, _P, _I64, C.POINTER(_I64), _V], C.c_int),
    "vbh_scene_last_touched": ([_V, _P, _I64, C.POINTER(_I64), _V], C.c_int),
    "vbh_scene_last_mc": ([_V, _P, _I64, C.POINTER(_I64), _V], C.c_int),
    "vbh_scene_read_blocks": ([_V, _P, _I64, _P, _P, _P, _P, _V], C.c_int),
    "vbh_scene_write_blocks": ([_V, _P, _I64, _P, _P, _P, C.c_uint32, _V], C.c_int),
    "vbh_scene_enable_timing": ([_V, _I32], C.c_int),
    "vbh_scene_timing": ([_V, C.POINTER(C.c_double), C.POINTER(_I64), C.POINTER(_I64), _V], C.c_int),
    "vbh_scene_log_entries": ([_V, _U64, _I64, _P, _P, _V], C.c_int),
    "vbh_scene_reset_blocks": ([_V, _P, _I64, C.c_uint32, _V], C.c_int),
    "vbh_mc_work_size": ([_I64], _I64),
    "vbh_mc_case": ([_I32, C.c_void_p], C.c_int),
    "vbh_mc_triangulate": ([_P, _P, _I64, C.c_float, _P, _P, _I64, _P, C.POINTER(_I64), _V], C.c_int),
    "vbh_cas_ceiling": ([_P, _I64, _I64, _U64, _P, _V], C.c_int),
    "vbh_check_division": ([_I64, _U64, C.c_int32, _P, _V], C.c_int),
    "vbh_mc_triangulate_static": ([_P, _P, _I64, C.c_float, _P, _P, _I64, C.POINTER(_I64), _V], C.c_int),
    "vbh_scene_visible_blocks": ([_V, C.POINTER(C.c_float), _P, _I64, C.POINTER(_I64), _V], C.c_int),
    "vbh_server_create": ([_V, C.POINTER(vbh_server_config), C.POINTER(_V)], C.c_int),
    "vbh_server_destroy": ([_V], None),
    "vbh_server_set_cursor": ([_V, _I32, _U64], C.c_int),
    "vbh_server_get_cursor": ([_V, _I32, C.POINTER(_U64)], C.c_int),
    "vbh_server_run": ([_V, C.POINTER(vbh_request), _I64, C.POINTER(vbh_frame_feed), _I64,
                        C.POINTER(vbh_request_result)], C.c_int),
    "vbh_diff_create": ([C.POINTER(vbh_params), _I32, C.POINTER(_V)], C.c_int),
    "vbh_diff_destroy": ([_V], None),
    "vbh_diff_forward": ([_V, _P, C.POINTER(C.c_float), _P, _P, _P, _I64, _P, _P, _V], C.c_int),
    "vbh_diff_backward": ([_V, _P, C.POINTER(C.c_float), _P, _P, _P, _I64, _P, _P, _P, _V], C.c_int),
}
STAGES = ("alloc", "integrate", "mc_mark", "mc_extract")


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is not built; run paper_1805_03709_amd/build.py "
                              "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes, fn.restype = args, res
        _lib = L
    return _lib


def lib():
    """The loaded C library with typed entry points (same names as include/vbh.h)."""
    return _load()


def exported_names():
    return list(SIGNATURES)


def _check(rc: int, what: str):
    if rc != VBH_OK:
        raise VbhError(rc, what)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, n=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on a HIP device")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, needs {n}")
    return C.c_void_p(t.data_ptr())


def _hptr(t, dtype, n, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.is_cuda:
        raise TypeError(f"{name} must be a CPU torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, needs {n}")
    return C.c_void_p(t.data_ptr())


def _poses_f32(poses, n):
    """n camera-to-world poses ([n][3][4] or [n][12], any float type, host or device) as a
    contiguous float32 [n][12] host array (each value rounded to nearest)."""
    if isinstance(poses, torch.Tensor):
        poses = poses.detach().cpu().numpy()
    a = np.asarray(poses, dtype=np.float64).reshape(n, -1)[:, :12]
    return np.ascontiguousarray(a, dtype=np.float32)


def _keys(keys):
    if keys.dim() != 2 or keys.shape[1] != 3:
        raise ValueError("keys must be int32 [n, 3]")
    return _ptr(keys, torch.int32, name="keys"), keys.shape[0]


class Map:
    """Concurrent int3 -> int32 hash map on the device (vbh_map_*)."""

    def __init__(self, slots: int, hash_kind: int = VBH_HASH_SPATIAL):
        self._L = lib()
        h = C.c_void_p()
        _check(lib().vbh_map_create(slots, hash_kind, C.byref(h)), "vbh_map_create")
        self.h, self.slots = h, slots

    def close(self):
        # the library object is held by the instance: module globals may already be gone
        # when this runs at interpreter exit
        L = getattr(self, "_L", None)
        if getattr(self, "h", None) and L is not None:
            L.vbh_map_destroy(self.h)
        self.h = None

    __del__ = close

    def vbh_insert(self, keys, vals, status=None):
        kp, n = _keys(keys)
        status = torch.empty(n, dtype=torch.int32, device=keys.device) if status is None else status
        _check(lib().vbh_insert(self.h, kp, _ptr(vals, torch.int32, n, "vals"), n,
                                _ptr(status, torch.int32, n, "status"), _stream()), "vbh_insert")
        return status

    def vbh_find(self, keys, out=None):
        kp, n = _keys(keys)
        out = torch.empty(n, dtype=torch.int32, device=keys.device) if out is None else out
        _check(lib().vbh_find(self.h, kp, n, _ptr(out, torch.int32, n, "out"), _stream()), "vbh_find")
        return out

    def vbh_erase(self, keys, status=None):
        kp, n = _keys(keys)
        status = torch.empty(n, dtype=torch.int32, device=keys.device) if status is None else status
        _check(lib().vbh_erase(self.h, kp, n, _ptr(status, torch.int32, n, "status"), _stream()), "vbh_erase")
        return status

    def vbh_apply(self, ops, keys, vals, out=None):
        kp, n = _keys(keys)
        out = torch.empty(n, dtype=torch.int32, device=keys.device) if out is None else out
        _check(lib().vbh_apply(self.h, _ptr(ops, torch.uint8, n, "ops"), kp, _ptr(vals, torch.int32, n, "vals"),
                               n, _ptr(out, torch.int32, n, "out"), _stream()), "vbh_apply")
        return out

    def vbh_map_size(self):
        live, tomb = C.c_int64(), C.c_int64()
        _check(lib().vbh_map_size(self.h, C.byref(live), C.byref(tomb), _stream()), "vbh_map_size")
        return live.value, tomb.value

    def vbh_size(self) -> int:
        n = C.c_int64()
        _check(lib().vbh_size(self.h, C.byref(n), _stream()), "vbh_size")
        return n.value

    def vbh_status(self) -> int:
        return lib().vbh_status(self.h, _stream())

    def vbh_map_export(self, device="cuda"):
        live, _ = self.vbh_map_size()
        keys = torch.empty((max(live, 1), 3), dtype=torch.int32, device=device)
        vals = torch.empty(max(live, 1), dtype=torch.int32, device=device)
        cnt = C.c_int64()
        _check(lib().vbh_map_export(self.h, _ptr(keys), _ptr(vals), live, C.byref(cnt), _stream()),
               "vbh_map_export")
        return keys[:cnt.value], vals[:cnt.value]

    def vbh_map_rebuild(self):
        _check(lib().vbh_map_rebuild(self.h, _stream()), "vbh_map_rebuild")

    def vbh_map_clear(self):
        _check(lib().vbh_map_clear(self.h, _stream()), "vbh_map_clear")

    def vbh_map_status(self) -> int:
        return int(lib().vbh_map_status(self.h, _stream()))


class ChainedMap(Map):
    """The paper's chained design behind the same calls (vbh_map_create_chained):
    `buckets` buckets plus `excess` linked-list entries."""

    def __init__(self, buckets: int, excess: int, hash_kind: int = VBH_HASH_SPATIAL):
        self._L = lib()
        h = C.c_void_p()
        _check(lib().vbh_map_create_chained(buckets, excess, hash_kind, C.byref(h)), "vbh_map_create_chained")
        self.h, self.slots, self.excess = h, buckets, excess


def vbh_cas_ceiling(words, n_ops: int, seed: int, won):
    """n_ops 64-bit CAS (expected 0) at pseudo-random words of the int64 tensor `words`
    (power-of-two length, zeroed); successes added to the int64 tensor `won`."""
    _check(lib().vbh_cas_ceiling(_ptr(words, torch.int64, name="words"), words.numel(), n_ops, seed,
                                 _ptr(won, torch.int64, 1, "won"), _stream()), "vbh_cas_ceiling")


def vbh_check_division(n: int, seed: int, all_ones: int, bad):
    """Count (into the int64 tensor `bad`) the n seeded operand pairs whose reciprocal-based
    projection quotient differs from the correctly rounded one."""
    _check(lib().vbh_check_division(n, seed, all_ones, _ptr(bad, torch.int64, 1, "bad"), _stream()),
           "vbh_check_division")


def vbh_mc_triangulate(keys, mcv, voxel_size: float):
    """Client triangles of MC voxel blocks (keys int32 [n,3], mcv int32/uint32 [n,512] on
    the device): (pos float32 [m,3,3], rgb uint8 [m,3])."""
    kp, n = _keys(keys)
    if mcv.dtype not in (torch.int32, torch.uint32) or mcv.numel() < 512 * n:
        raise TypeError("mcv must be a 32-bit [n, 512] device tensor")
    mp = _ptr(mcv, None, 512 * n, "mcv")
    work = torch.empty(max(int(lib().vbh_mc_work_size(n)), 1), dtype=torch.int64, device=keys.device)
    cnt = C.c_int64()
    _check(lib().vbh_mc_triangulate(kp, mp, n, voxel_size, None, None, 0, _ptr(work), C.byref(cnt), _stream()),
           "vbh_mc_triangulate")
    m = cnt.value
    pos = torch.empty((max(m, 1), 3, 3), dtype=torch.float32, device=keys.device)
    rgb = torch.empty((max(m, 1), 3), dtype=torch.uint8, device=keys.device)
    _check(lib().vbh_mc_triangulate(kp, mp, n, voxel_size, _ptr(pos), _ptr(rgb), m, _ptr(work), C.byref(cnt),
                                    _stream()), "vbh_mc_triangulate")
    return pos[:m], rgb[:m]


def make_params(vol, cam, hash_kind: int = VBH_HASH_SPATIAL) -> vbh_params:
    return vbh_params(vol.slots, vol.pool_blocks, vol.log_capacity, vol.voxel_size, vol.trunc,
                      cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, vol.depth_min,
                      vol.depth_max, hash_kind)


class Scene:
    """Block-hashed TSDF volume with MC voxel pool and update log (vbh_scene_*)."""

    def __init__(self, params: vbh_params):
        self.params = params
        self._L = lib()
        h = C.c_void_p()
        _check(lib().vbh_scene_create(C.byref(params), C.byref(h)), "vbh_scene_create")
        self.h = h

    def close(self):
        # the library object is held by the instance: module globals may already be gone
        # when this runs at interpreter exit
        L = getattr(self, "_L", None)
        if getattr(self, "h", None) and L is not None:
            L.vbh_scene_destroy(self.h)
        self.h = None

    __del__ = close

    def vbh_integrate_frame(self, depth, rgb, pose_c2w, frame_id: int):
        p = self.params
        n = p.width * p.height
        P = _poses_f32(pose_c2w, 1)
        pose = P.ctypes.data_as(C.POINTER(C.c_float))
        _check(lib().vbh_integrate_frame(self.h, _ptr(depth, torch.float32, n, "depth"),
                                         _ptr(rgb, torch.uint8, 3 * n, "rgb"), pose, frame_id, _stream()),
               "vbh_integrate_frame")

    def vbh_integrate_blocks(self, keys, depth, rgb, pose_c2w, frame_id: int):
        kp, nk = _keys(keys)
        p = self.params
        n = p.width * p.height
        P = _poses_f32(pose_c2w, 1)
        _check(lib().vbh_integrate_blocks(self.h, kp, nk, _ptr(depth, torch.float32, n, "depth"),
                                          _ptr(rgb, torch.uint8, 3 * n, "rgb"), P.ctypes.data_as(C.POINTER(C.c_float)),
                                          frame_id, _stream()),
               "vbh_integrate_blocks")

    def vbh_integrate_frames(self, depth, rgb, poses_c2w, first_frame_id: int):
        """Fuse frames depth[i] (rgb[i], poses_c2w[i]) as ids first_frame_id + i."""
        p = self.params
        n = int(depth.shape[0]) if depth is not None else 0
        hw = p.width * p.height
        P = _poses_f32(poses_c2w, n) if n > 0 else np.zeros((1, 12), np.float32)
        poses = P.ctypes.data_as(C.POINTER(C.c_float))
        _check(lib().vbh_integrate_frames(self.h, _ptr(depth, torch.float32, n * hw, "depth"),
                                          _ptr(rgb, torch.uint8, 3 * n * hw, "rgb"), poses, first_frame_id, n,
                                          _stream()), "vbh_integrate_frames")

    def vbh_integrate_frames_host(self, depth, rgb, poses_c2w, first_frame_id: int):
        """vbh_integrate_frames for CPU tensors (pin_memory() ones overlap the uploads)."""
        p = self.params
        n = int(depth.shape[0]) if depth is not None else 0
        hw = p.width * p.height
        P = _poses_f32(poses_c2w, n) if n > 0 else np.zeros((1, 12), np.float32)
        _check(lib().vbh_integrate_frames_host(self.h, _hptr(depth, torch.float32, n * hw, "depth"),
                                               _hptr(rgb, torch.uint8, 3 * n * hw, "rgb"),
                                               P.ctypes.data_as(C.POINTER(C.c_float)), first_frame_id, n, _stream()),
               "vbh_integrate_frames_host")

    def vbh_extract_mc_indices(self, keys, with_rgb=True):
        kp, n = _keys(keys)
        mc = torch.empty((n, 512), dtype=torch.uint8, device=keys.device)
        rgb = torch.empty((n, 512, 3), dtype=torch.uint8, device=keys.device) if with_rgb else None
        _check(lib().vbh_extract_mc_indices(self.h, kp, n, _ptr(mc), _ptr(rgb), _stream()),
               "vbh_extract_mc_indices")
        return mc, rgb

    def vbh_extract_mc_all(self, cap, with_rgb=True, device="cuda"):
        """Every allocated block (up to cap): (keys int32 [m,3], MC uint8 [m,512], RGB or None,
        allocated count)."""
        keys = torch.empty((max(cap, 1), 3), dtype=torch.int32, device=device)
        mc = torch.empty((max(cap, 1), 512), dtype=torch.uint8, device=device)
        rgb = torch.empty((max(cap, 1), 512, 3), dtype=torch.uint8, device=device) if with_rgb else None
        n = C.c_int64()
        _check(lib().vbh_extract_mc_all(self.h, _ptr(keys), cap, _ptr(mc), _ptr(rgb), C.byref(n), _stream()),
               "vbh_extract_mc_all")
        m = min(cap, n.value)
        return keys[:m], mc[:m], (rgb[:m] if rgb is not None else None), n.value

    def vbh_status(self) -> int:
        return lib().vbh_status(self.h, _stream())

    def vbh_stored_mc(self, keys, with_rgb=True):
        kp, n = _keys(keys)
        mc = torch.empty((n, 512), dtype=torch.uint8, device=keys.device)
        rgb = torch.empty((n, 512, 3), dtype=torch.uint8, device=keys.device) if with_rgb else None
        _check(lib().vbh_stored_mc(self.h, kp, n, _ptr(mc), _ptr(rgb), _stream()), "vbh_stored_mc")
        return mc, rgb

    def vbh_updated_blocks_since(self, cursor: int, cap: int, device="cuda"):
        keys = torch.empty((max(cap, 1), 3), dtype=torch.int32, device=device)
        meta = torch.zeros(2, dtype=torch.int64, device=device)  # [count, next cursor]
        _check(lib().vbh_updated_blocks_since(self.h, cursor, cap, _ptr(keys), C.c_void_p(meta.data_ptr()),
                                              C.c_void_p(meta.data_ptr() + 8), _stream()),
               "vbh_updated_blocks_since")
        return keys, meta

    def vbh_scene_status(self) -> int:
        return int(lib().vbh_scene_status(self.h, _stream()))

    def vbh_scene_stats(self) -> dict:
        st = vbh_stats()
        _check(lib().vbh_scene_stats(self.h, C.byref(st), _stream()), "vbh_scene_stats")
        return st.as_dict()

    def _keylist(self, fn, name, device):
        cnt = C.c_int64()
        _check(fn(self.h, None, 0, C.byref(cnt), _stream()), name)
        keys = torch.empty((max(cnt.value, 1), 3), dtype=torch.int32, device=device)
        _check(fn(self.h, _ptr(keys), cnt.value, C.byref(cnt), _stream()), name)
        return keys[:cnt.value]

    def vbh_scene_export_blocks(self, device="cuda"):
        return self._keylist(lib().vbh_scene_export_blocks, "vbh_scene_export_blocks", device)

    def vbh_scene_last_touched(self, device="cuda"):
        return self._keylist(lib().vbh_scene_last_touched, "vbh_scene_last_touched", device)

    def vbh_scene_last_mc(self, device="cuda"):
        return self._keylist(lib().vbh_scene_last_mc, "vbh_scene_last_mc", device)

    def vbh_scene_read_blocks(self, keys):
        kp, n = _keys(keys)
        F = torch.empty((n, 512), dtype=torch.float32, device=keys.device)
        W = torch.empty((n, 512), dtype=torch.uint8, device=keys.device)
        rgb = torch.empty((n, 512, 3), dtype=torch.uint8, device=keys.device)
        found = torch.empty(n, dtype=torch.int32, device=keys.device)
        _check(lib().vbh_scene_read_blocks(self.h, kp, n, _ptr(F), _ptr(W), _ptr(rgb), _ptr(found), _stream()),
               "vbh_scene_read_blocks")
        return F, W, rgb, found

    def vbh_scene_reset_blocks(self, keys, frame_id: int):
        kp, n = _keys(keys)
        _check(lib().vbh_scene_reset_blocks(self.h, kp, n, frame_id, _stream()), "vbh_scene_reset_blocks")

    def vbh_scene_visible_blocks(self, pose_c2w, device="cuda"):
        P = _poses_f32(pose_c2w, 1)
        pose = P.ctypes.data_as(C.POINTER(C.c_float))
        cnt = C.c_int64()
        _check(lib().vbh_scene_visible_blocks(self.h, pose, None, 0, C.byref(cnt), _stream()),
               "vbh_scene_visible_blocks")
        keys = torch.empty((max(cnt.value, 1), 3), dtype=torch.int32, device=device)
        _check(lib().vbh_scene_visible_blocks(self.h, pose, _ptr(keys), cnt.value, C.byref(cnt), _stream()),
               "vbh_scene_visible_blocks")
        return keys[:cnt.value]

    def vbh_scene_log_entries(self, start: int, n: int, device="cuda"):
        fr = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        keys = torch.empty((max(n, 1), 3), dtype=torch.int32, device=device)
        _check(lib().vbh_scene_log_entries(self.h, start, n, _ptr(fr), _ptr(keys), _stream()),
               "vbh_scene_log_entries")
        return fr[:n], keys[:n]

    def vbh_scene_enable_timing(self, period: int = 1):
        """Time the kernels of every `period`-th update (0 turns timing off)."""
        _check(lib().vbh_scene_enable_timing(self.h, int(period)), "vbh_scene_enable_timing")

    def vbh_scene_timing(self, with_blocks=False):
        """{stage: summed kernel ms}, frames measured (synchronising; resets); with_blocks
        also returns (touched blocks, MC-set blocks) of exactly the measured updates."""
        ms = (C.c_double * len(STAGES))()
        frames = C.c_int64()
        blk = (C.c_int64 * 2)()
        _check(lib().vbh_scene_timing(self.h, ms, C.byref(frames), blk, _stream()), "vbh_scene_timing")
        if with_blocks:
            return dict(zip(STAGES, list(ms))), frames.value, (blk[0], blk[1])
        return dict(zip(STAGES, list(ms))), frames.value

    def vbh_scene_write_blocks(self, keys, F, W, rgb, frame_id: int):
        kp, n = _keys(keys)
        _check(lib().vbh_scene_write_blocks(self.h, kp, n, _ptr(F, torch.float32, 512 * n, "F"),
                                            _ptr(W, torch.uint8, 512 * n, "W"),
                                            _ptr(rgb, torch.uint8, 1536 * n, "rgb"), frame_id, _stream()),
               "vbh_scene_write_blocks")


class Server:
    """Serving loop over a scene (vbh_server_*)."""

    def __init__(self, scene: Scene, arena_bytes: int, max_inflight: int = 256, n_streams: int = 4,
                 n_clients: int = 64, max_batch: int = 64, mode: int = 0, workgroups: int = 0):
        """mode 0: rounds of kernels on n_streams streams; mode 1: one persistent launch per
        scene version with n_streams teams (1..4) of `workgroups` workgroups in all."""
        self.cfg = vbh_server_config(arena_bytes, max_inflight, n_streams, n_clients, max_batch, mode, workgroups)
        self._L = lib()
        h = C.c_void_p()
        _check(lib().vbh_server_create(scene.h, C.byref(self.cfg), C.byref(h)), "vbh_server_create")
        self.h, self.scene = h, scene

    def close(self):
        # the library object is held by the instance: module globals may already be gone
        # when this runs at interpreter exit
        L = getattr(self, "_L", None)
        if getattr(self, "h", None) and L is not None:
            L.vbh_server_destroy(self.h)
        self.h = None

    __del__ = close

    def vbh_server_set_cursor(self, client: int, cursor: int):
        _check(lib().vbh_server_set_cursor(self.h, client, cursor), "vbh_server_set_cursor")

    def vbh_server_get_cursor(self, client: int) -> int:
        c = C.c_uint64()
        _check(lib().vbh_server_get_cursor(self.h, client, C.byref(c)), "vbh_server_get_cursor")
        return c.value

    def vbh_server_run(self, clients, limits, arrivals, outputs=None, frames=None):
        """clients/limits/arrivals: sequences (arrivals non-decreasing, seconds).  outputs:
        optional list of (keys int32 [limit,3], mc int32 [limit,512]) device tensors per
        request.  frames: optional list of (depth, rgb or None, pose 3x4, time_s, frame_id).
        Returns a numpy structured array of results."""
        n = len(clients)
        reqs = (vbh_request * max(n, 1))()
        for i in range(n):
            reqs[i].client, reqs[i].limit, reqs[i].arrival_s = int(clients[i]), int(limits[i]), float(arrivals[i])
            if outputs is not None and outputs[i] is not None:
                k, m = outputs[i]
                reqs[i].d_keys_out = _ptr(k, torch.int32, 3 * int(limits[i]))
                reqs[i].d_mc_out = _ptr(m, torch.int32, 512 * int(limits[i]))
        frames = frames or []
        feed = (vbh_frame_feed * max(len(frames), 1))()
        for i, (d, c, pose, t, fid) in enumerate(frames):
            feed[i].d_depth = _ptr(d, torch.float32)
            feed[i].d_rgb = _ptr(c, torch.uint8) if c is not None else None
            feed[i].pose_c2w[:] = _poses_f32(pose, 1).reshape(-1).tolist()
            feed[i].time_s, feed[i].frame_id = float(t), int(fid)
        res = (vbh_request_result * max(n, 1))()
        torch.cuda.synchronize()
        _check(lib().vbh_server_run(self.h, reqs, n, feed, len(frames), res), "vbh_server_run")
        import numpy as np
        dt = np.dtype([(f, np.float64 if t is C.c_double else np.int64) for f, t in vbh_request_result._fields_])
        out = np.zeros(n, dt)
        for i in range(n):
            for f, _ in vbh_request_result._fields_:
                out[f][i] = getattr(res[i], f)
        return out
