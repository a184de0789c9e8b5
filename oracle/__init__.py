"""ctypes front end of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package; the HIP product path never does.  All arrays are host numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

ABSENT = -(1 << 31)
_lib = None


_SIG = None


def _signatures():
    vp, i64, i32p, u8p, f32p, f64p = C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p
    sig = {
        "orc_map_new": ([], vp), "orc_map_free": ([vp], None),
        "orc_map_insert": ([vp, i32p, i32p, i64, i32p], C.c_int),
        "orc_map_find": ([vp, i32p, i64, i32p], C.c_int),
        "orc_map_erase": ([vp, i32p, i64, i32p], C.c_int),
        "orc_map_apply": ([vp, u8p, i32p, i32p, i64, i32p], C.c_int),
        "orc_map_size": ([vp], i64),
        "orc_map_export": ([vp, i32p, i32p, i64], i64),
        "orc_scene_new": ([vp], vp), "orc_scene_free": ([vp], None),
        "orc_integrate_frame": ([vp, f32p, u8p, f32p, C.c_uint32], C.c_int),
        "orc_integrate_blocks": ([vp, i32p, i64, f32p, u8p, f32p, C.c_uint32], C.c_int),
        "orc_last_touched": ([vp, i32p, i64], i64),
        "orc_last_new": ([vp, i32p, i64], i64),
        "orc_last_mc_updated": ([vp, i32p, i64], i64),
        "orc_n_blocks": ([vp], i64),
        "orc_export_blocks": ([vp, i32p, i64], i64),
        "orc_read_blocks": ([vp, i32p, i64, f64p, u8p, u8p, i32p], C.c_int),
        "orc_write_blocks": ([vp, i32p, i64, f32p, u8p, u8p, C.c_uint32], C.c_int),
        "orc_reset_blocks": ([vp, i32p, i64, C.c_uint32, C.c_void_p], C.c_int),
        "orc_visible_blocks": ([vp, f32p, i32p, i64], i64),
        "orc_mc_triangles": ([i32p, C.c_void_p, i64, C.c_float, f32p, u8p, i64], i64),
        "orc_extract_mc": ([vp, i32p, i64, u8p, u8p], C.c_int),
        "orc_stored_mc": ([vp, i32p, i64, u8p, u8p], C.c_int),
        "orc_updated_since": ([vp, C.c_uint64, i64, i32p, C.c_void_p], i64),
        "orc_log_length": ([vp], C.c_uint64),
        "orc_scene_error": ([vp], C.c_int),
        "orc_streams_new": ([vp, C.c_int32], vp), "orc_streams_free": ([vp], None),
        "orc_streams_sync": ([vp], i64),
        "orc_streams_reconnect": ([vp, C.c_int32], C.c_int),
        "orc_streams_pending": ([vp, C.c_int32, i32p, C.c_void_p, i64], i64),
        "orc_streams_serve": ([vp, C.c_int32, i64, i32p], i64),
        "orc_streams_take": ([vp, C.c_int32, i64, i32p, i64], C.c_int),
        "orc_diff_new": ([vp], vp), "orc_diff_free": ([vp], None),
        "orc_diff_loss": ([vp, f64p, C.c_double, f64p], C.c_double),
        "orc_diff_grad": ([vp, f64p, f64p], C.c_int),
        "orc_diff_info": ([vp, C.c_void_p, C.c_void_p, f64p], i64),
    }
    return sig


def load(path: str):
    """Loads an oracle library built from these sources at `path` with typed entry points
    (the default one is lib(); tests also load variants with planted mistakes)."""
    L = C.CDLL(path)
    for name, (args, res) in _signatures().items():
        if not hasattr(L, name):
            raise RuntimeError(f"oracle library {path} lacks {name}")
        fn = getattr(L, name)
        fn.argtypes, fn.restype = args, res
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = load(LIB)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _keys(keys):
    k = np.ascontiguousarray(keys, dtype=np.int32).reshape(-1, 3)
    return k, k.shape[0]


class Map:
    """std::unordered_map semantics; batches run serially in index order."""

    def __init__(self, L=None):
        self.L = L or lib()
        self.h = self.L.orc_map_new()

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_map_free(self.h)
            self.h = None

    def insert(self, keys, vals):
        k, n = _keys(keys)
        v = np.ascontiguousarray(vals, np.int32)
        out = np.empty(n, np.int32)
        rc = self.L.orc_map_insert(self.h, _p(k), _p(v), n, _p(out))
        return out, rc

    def find(self, keys):
        k, n = _keys(keys)
        out = np.empty(n, np.int32)
        self.L.orc_map_find(self.h, _p(k), n, _p(out))
        return out

    def erase(self, keys):
        k, n = _keys(keys)
        out = np.empty(n, np.int32)
        rc = self.L.orc_map_erase(self.h, _p(k), n, _p(out))
        return out, rc

    def apply(self, ops, keys, vals):
        k, n = _keys(keys)
        o = np.ascontiguousarray(ops, np.uint8)
        v = np.ascontiguousarray(vals, np.int32)
        out = np.empty(n, np.int32)
        rc = self.L.orc_map_apply(self.h, _p(o), _p(k), _p(v), n, _p(out))
        return out, rc

    def size(self):
        return int(self.L.orc_map_size(self.h))

    def export(self):
        n = self.size()
        k = np.empty((n, 3), np.int32)
        v = np.empty(n, np.int32)
        self.L.orc_map_export(self.h, _p(k), _p(v), n)
        return k, v


class OrcParams(C.Structure):
    _fields_ = [("pool_blocks", C.c_int64), ("log_capacity", C.c_int64),
                ("voxel_size", C.c_float), ("trunc", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("depth_min", C.c_float), ("depth_max", C.c_float)]


def make_params(vol, cam) -> OrcParams:
    return OrcParams(vol.pool_blocks, vol.log_capacity, vol.voxel_size, vol.trunc, cam.width,
                     cam.height, cam.fx, cam.fy, cam.cx, cam.cy, vol.depth_min, vol.depth_max)


def pose32(pose) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(pose, np.float64).reshape(3, 4), np.float32)


class Scene:
    """Block-hashed TSDF volume: allocation, integration, MC voxels, update log."""

    def __init__(self, vol, cam, L=None):
        self.L = L or lib()
        self.params = make_params(vol, cam)
        self.h = self.L.orc_scene_new(C.byref(self.params))
        if not self.h:
            raise ValueError("invalid oracle scene parameters")

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_scene_free(self.h)
            self.h = None

    def integrate(self, depth, rgb, pose, frame_id: int) -> int:
        d = np.ascontiguousarray(depth, np.float32)
        c = None if rgb is None else np.ascontiguousarray(rgb, np.uint8)
        P = pose32(pose)
        return self.L.orc_integrate_frame(self.h, _p(d), _p(c), _p(P), frame_id)

    def integrate_blocks(self, keys, depth, rgb, pose, frame_id: int) -> int:
        k, n = _keys(keys)
        d = np.ascontiguousarray(depth, np.float32)
        c = None if rgb is None else np.ascontiguousarray(rgb, np.uint8)
        P = pose32(pose)
        return int(self.L.orc_integrate_blocks(self.h, _p(k) if n else None, n, _p(d), _p(c), _p(P), frame_id))

    def _keylist(self, fn):
        n = fn(self.h, None, 0)
        k = np.empty((n, 3), np.int32)
        fn(self.h, _p(k), n)
        return k

    def last_touched(self):
        return self._keylist(self.L.orc_last_touched)

    def last_new(self):
        return self._keylist(self.L.orc_last_new)

    def last_mc_updated(self):
        return self._keylist(self.L.orc_last_mc_updated)

    def blocks(self):
        return self._keylist(self.L.orc_export_blocks)

    def n_blocks(self):
        return int(self.L.orc_n_blocks(self.h))

    def read(self, keys):
        k, n = _keys(keys)
        F = np.empty((n, 512), np.float64)
        W = np.empty((n, 512), np.uint8)
        rgb = np.empty((n, 512, 3), np.uint8)
        found = np.empty(n, np.int32)
        self.L.orc_read_blocks(self.h, _p(k), n, _p(F), _p(W), _p(rgb), _p(found))
        return F, W, rgb, found

    def write(self, keys, F, W, rgb, frame_id: int) -> int:
        k, n = _keys(keys)
        F = np.ascontiguousarray(F, np.float32)
        W = np.ascontiguousarray(W, np.uint8)
        c = None if rgb is None else np.ascontiguousarray(rgb, np.uint8)
        return self.L.orc_write_blocks(self.h, _p(k), n, _p(F), _p(W), _p(c), frame_id)

    def reset_blocks(self, keys, frame_id: int):
        """Returns (status, number of distinct blocks reset)."""
        k, n = _keys(keys)
        cnt = C.c_int64()
        rc = self.L.orc_reset_blocks(self.h, _p(k), n, frame_id, C.byref(cnt))
        return rc, cnt.value

    def visible_blocks(self, pose):
        P = np.ascontiguousarray(np.asarray(pose, np.float32).reshape(-1)[:12])
        n = self.L.orc_visible_blocks(self.h, _p(P), None, 0)
        k = np.empty((max(n, 1), 3), np.int32)
        self.L.orc_visible_blocks(self.h, _p(P), _p(k), n)
        return k[:n]

    def extract_mc(self, keys):
        k, n = _keys(keys)
        mc = np.empty((n, 512), np.uint8)
        rgb = np.empty((n, 512, 3), np.uint8)
        self.L.orc_extract_mc(self.h, _p(k), n, _p(mc), _p(rgb))
        return mc, rgb

    def stored_mc(self, keys):
        k, n = _keys(keys)
        mc = np.empty((n, 512), np.uint8)
        rgb = np.empty((n, 512, 3), np.uint8)
        self.L.orc_stored_mc(self.h, _p(k), n, _p(mc), _p(rgb))
        return mc, rgb

    def updated_since(self, cursor: int, cap: int):
        k = np.empty((max(cap, 0), 3), np.int32)
        nxt = np.zeros(1, np.uint64)
        n = self.L.orc_updated_since(self.h, cursor, cap, _p(k), nxt.ctypes.data)
        return k[:n], int(nxt[0])

    def log_length(self):
        return int(self.L.orc_log_length(self.h))

    def error(self):
        return int(self.L.orc_scene_error(self.h))


SERVE_ECOUNT, SERVE_EDUP, SERVE_ENOTPENDING, SERVE_EORDER = -20, -21, -22, -23


class Streams:
    """Per-client stream sets of a Scene (Sec. 4.2): the blocks updated since they were
    last sent to each client, oldest updates served first."""

    def __init__(self, scene: Scene, n_clients: int):
        self.L, self.scene = scene.L, scene  # the scene must outlive the streams
        self.h = self.L.orc_streams_new(scene.h, n_clients)
        if not self.h:
            raise ValueError("invalid stream parameters")

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_streams_free(self.h)
            self.h = None

    def sync(self) -> int:
        """Absorb the scene's update-log entries appended since the last call."""
        return int(self.L.orc_streams_sync(self.h))

    def reconnect(self, client: int):
        assert self.L.orc_streams_reconnect(self.h, client) == 0

    def pending(self, client: int):
        """(keys int32 [n,3], frames uint32 [n]) in (update frame, packed key) order."""
        n = int(self.L.orc_streams_pending(self.h, client, None, None, 0))
        k = np.empty((max(n, 1), 3), np.int32)
        f = np.empty(max(n, 1), np.uint32)
        self.L.orc_streams_pending(self.h, client, _p(k), f.ctypes.data, n)
        return k[:n], f[:n]

    def serve(self, client: int, limit: int):
        k = np.empty((max(limit, 1), 3), np.int32)
        n = int(self.L.orc_streams_serve(self.h, client, limit, _p(k)))
        assert n >= 0
        return k[:n]

    def take(self, client: int, limit: int, keys) -> int:
        """0 if `keys` is a valid answer (then removed from the client's set), else an
        SERVE_E* code and the set is unchanged."""
        k, n = _keys(keys)
        return int(self.L.orc_streams_take(self.h, client, limit, _p(k) if n else None, n))


class DiffProblemStruct(C.Structure):
    _fields_ = [("p", OrcParams), ("n_frames", C.c_int32), ("depth", C.c_void_p), ("poses", C.c_void_p),
                ("n_samples", C.c_int64), ("sample_frame", C.c_void_p), ("sample_pixel", C.c_void_p),
                ("xi_ref", C.c_void_p)]


class Diff:
    """Frozen-branch float64 forward and gradient of L = sum_k F_tri(x_k)^2 (see diff.cpp)."""

    def __init__(self, vol, cam, depth, poses, sample_frame, sample_pixel, L=None, xi_ref=None):
        """poses: base poses T0 [F,3,4]; xi_ref [F,6] (optional): the reference point
        T_f = Exp(xi_ref_f) T0_f at which the branches freeze and the gradient is taken."""
        self.L = L or lib()
        self.depth = np.ascontiguousarray(depth, np.float32)
        self.poses = np.ascontiguousarray(np.asarray(poses, np.float64).reshape(-1, 3, 4), np.float32)
        self.sf = np.ascontiguousarray(sample_frame, np.int32)
        self.sp = np.ascontiguousarray(sample_pixel, np.int32)
        self.F, self.HW = self.depth.shape[0], cam.width * cam.height
        self.xi_ref = (np.zeros((self.F, 6)) if xi_ref is None
                       else np.ascontiguousarray(np.asarray(xi_ref, np.float64).reshape(self.F, 6)))
        prob = DiffProblemStruct(make_params(vol, cam), self.F, self.depth.ctypes.data, self.poses.ctypes.data,
                                 self.sf.size, self.sf.ctypes.data, self.sp.ctypes.data,
                                 None if xi_ref is None else self.xi_ref.ctypes.data)
        self.h = self.L.orc_diff_new(C.byref(prob))
        if not self.h:
            raise ValueError("invalid differentiable problem")

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_diff_free(self.h)
            self.h = None

    def loss(self, d_depth=None, scale=0.0, xi=None):
        dd = None if d_depth is None else np.ascontiguousarray(d_depth, np.float64)
        x = None if xi is None else np.ascontiguousarray(xi, np.float64)
        return float(self.L.orc_diff_loss(self.h, _p(dd), scale, _p(x)))

    def grad(self):
        gD = np.empty(self.F * self.HW, np.float64)
        gx = np.empty(self.F * 6, np.float64)
        self.L.orc_diff_grad(self.h, _p(gD), _p(gx))
        return gD.reshape(self.F, -1), gx.reshape(self.F, 6)

    def info(self):
        kept, ngv = C.c_int64(), C.c_int64()
        f = np.empty(self.sf.size, np.float64)
        nb = self.L.orc_diff_info(self.h, C.byref(kept), C.byref(ngv), _p(f))
        return {"blocks": int(nb), "kept": kept.value, "grad_voxels": ngv.value, "f_samples": f}

    # Central differences with step h.  points=3: (L(h) - L(-h)) / 2h; points=5 adds one
    # Richardson step, (8 (L(h) - L(-h)) - (L(2h) - L(-2h))) / 12h, removing the O(h^2) term.
    @staticmethod
    def _central(fn, h, points):
        d1 = (fn(h) - fn(-h)) / (2 * h)
        if points == 3:
            return d1
        d2 = (fn(2 * h) - fn(-2 * h)) / (4 * h)
        return (4 * d1 - d2) / 3

    def fd_pose(self, f, a, h=1e-4, points=5):
        def fn(t):
            xi = self.xi_ref.copy()
            xi[f, a] += t
            return self.loss(xi=xi)
        return self._central(fn, h, points)

    def fd_depth(self, f, pix, h=1e-4, points=5):
        v = np.zeros((self.F, self.HW))
        v[f, pix] = 1.0
        return self._central(lambda t: self.loss(v, t), h, points)

    def fd_direction(self, v_depth, v_xi, h=1e-4, points=5):
        return self._central(lambda t: self.loss(v_depth, t, self.xi_ref + t * v_xi), h, points)


def rel_err(g, g_ref, scale_ref=None):
    """|g - g_ref| / max(|g_ref|, 1e-3 max|g_ref|) elementwise."""
    g, g_ref = np.asarray(g, np.float64), np.asarray(g_ref, np.float64)
    s = np.abs(g_ref).max() if scale_ref is None else scale_ref
    return np.abs(g - g_ref) / np.maximum(np.abs(g_ref), 1e-3 * s)


def mc_triangles(keys, mcv, voxel_size, L=None):
    """Client triangulation of MC voxel blocks: (pos float32 [m,3,3], rgb uint8 [m,3])."""
    L = L or lib()
    k, n = _keys(keys)
    v = np.ascontiguousarray(mcv).view(np.uint32).reshape(n, 512)
    m = L.orc_mc_triangles(_p(k), v.ctypes.data, n, voxel_size, None, None, 0)
    pos = np.empty((max(m, 1), 3, 3), np.float32)
    rgb = np.empty((max(m, 1), 3), np.uint8)
    L.orc_mc_triangles(_p(k), v.ctypes.data, n, voxel_size, _p(pos), _p(rgb), m)
    return pos[:m], rgb[:m]
