"""Streaming packets of the server (Sec. 4.2): the bytes a request's answer is sent as.

An MC packet holds, per block, its int32 (x, y, z) key and its 512 MC voxels of 4 bytes
(case index | R << 8 | G << 16 | B << 24, x fastest), which is the paper's compact voxel
representation; a TSDF packet holds, per block, the key and 512 TSDF voxels of 12 bytes
(float32 distance, float32 weight, RGB8, one pad byte), the standard voxel-hashing
representation the paper compares against.  Packets are compressed losslessly with zstd
(Sec. 4.1-4.2), through the system's libzstd.
"""
from __future__ import annotations

import ctypes as C
import ctypes.util

import numpy as np

_zstd = None


def _lib():
    global _zstd
    if _zstd is None:
        name = ctypes.util.find_library("zstd") or "libzstd.so.1"
        L = C.CDLL(name)  # raises if the system has no libzstd
        L.ZSTD_compressBound.argtypes, L.ZSTD_compressBound.restype = [C.c_size_t], C.c_size_t
        L.ZSTD_compress.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t, C.c_int]
        L.ZSTD_compress.restype = C.c_size_t
        L.ZSTD_decompress.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t]
        L.ZSTD_decompress.restype = C.c_size_t
        L.ZSTD_isError.argtypes, L.ZSTD_isError.restype = [C.c_size_t], C.c_uint
        _zstd = L
    return _zstd


def zstd_compress(data, level: int = 1) -> bytes:
    src = np.ascontiguousarray(np.frombuffer(memoryview(data).cast("B"), dtype=np.uint8))
    L = _lib()
    cap = L.ZSTD_compressBound(src.size)
    dst = np.empty(cap, np.uint8)
    n = L.ZSTD_compress(dst.ctypes.data, cap, src.ctypes.data, src.size, level)
    if L.ZSTD_isError(n):
        raise RuntimeError("ZSTD_compress failed")
    return dst[:n].tobytes()


def zstd_decompress(data: bytes, size: int) -> bytes:
    src = np.frombuffer(data, dtype=np.uint8)
    dst = np.empty(max(size, 1), np.uint8)
    n = _lib().ZSTD_decompress(dst.ctypes.data, size, src.ctypes.data, src.size)
    if _lib().ZSTD_isError(n) or n != size:
        raise RuntimeError("ZSTD_decompress failed")
    return dst[:size].tobytes()


def mc_packet(keys: np.ndarray, mcv: np.ndarray) -> bytes:
    """keys int32 [n,3], mcv uint32/int32 [n,512] packed MC voxels -> packet bytes."""
    keys = np.ascontiguousarray(keys, np.int32).reshape(-1, 3)
    mcv = np.ascontiguousarray(mcv).view(np.uint32).reshape(-1, 512)
    rec = np.empty(keys.shape[0], dtype=[("key", "<i4", 3), ("mc", "<u4", 512)])
    rec["key"], rec["mc"] = keys, mcv
    return rec.tobytes()


def tsdf_packet(keys: np.ndarray, F: np.ndarray, W: np.ndarray, rgb: np.ndarray) -> bytes:
    """keys int32 [n,3], F float32 [n,512], W uint8 [n,512], rgb uint8 [n,512,3] -> packet
    bytes of 12-byte TSDF voxels."""
    n = keys.shape[0]
    vox = np.zeros((n, 512), dtype=[("f", "<f4"), ("w", "<f4"), ("rgb", "u1", 3), ("pad", "u1")])
    vox["f"], vox["w"], vox["rgb"] = F, W.astype(np.float32), rgb
    rec = np.empty(n, dtype=[("key", "<i4", 3), ("vox", vox.dtype, 512)])
    rec["key"], rec["vox"] = np.ascontiguousarray(keys, np.int32).reshape(-1, 3), vox
    return rec.tobytes()


MC_BLOCK_BYTES = 12 + 512 * 4
TSDF_BLOCK_BYTES = 12 + 512 * 12
