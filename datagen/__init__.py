"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds scene geometry, ray casting, sensor noise, camera trajectories and
hash-key/op streams.  It contains none of the reconstruction method's own arithmetic
(no hashing, block allocation, fusion or Marching Cubes): both the CPU oracle and the
HIP path consume the exact bytes produced here.
"""
from .scenes import (Camera, Scene, box_room_scene, room_of_boxes_scene, look_at,
                     raycast, render_frames, kinect_noise, trajectory_c3, scene_sdf)
from .hashgen import (pack_key, unpack_key, fmix64, value_of, bulk_keys,
                      mixed_batches, adversarial_batch, OP_INSERT, OP_FIND, OP_ERASE)
from . import configs

__all__ = [
    "Camera", "Scene", "box_room_scene", "room_of_boxes_scene", "look_at", "raycast",
    "render_frames", "kinect_noise", "trajectory_c3", "scene_sdf", "pack_key",
    "unpack_key", "fmix64", "value_of", "bulk_keys", "mixed_batches",
    "adversarial_batch", "OP_INSERT", "OP_FIND", "OP_ERASE", "configs",
]
