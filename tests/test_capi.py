"""The C-ABI library loads and exports every symbol include/vbh.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vbh_[a-z0-9_]+)\s*\(", text)))


def libpath():
    from paper_1805_03709_amd.build import LIB
    if not os.path.exists(LIB):
        pytest.skip("libvbh.so not built")
    return LIB


def test_every_declared_symbol_is_exported():
    L = ctypes.CDLL(libpath())
    names = declared("vbh.h")
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1805_03709_amd import binding
    assert set(declared("vbh.h")) == set(binding.exported_names())


def test_host_side_argument_errors_need_no_gpu():
    from paper_1805_03709_amd import binding
    L = binding.lib()
    assert L.vbh_version() == 1
    assert L.vbh_strerror(-5) == b"voxel block pool exhausted"
    h = ctypes.c_void_p()
    # non-power-of-two slot counts and bad hash kinds are rejected before any HIP call
    assert L.vbh_map_create(1000, 0, ctypes.byref(h)) == binding.VBH_EINVAL
    assert L.vbh_map_create(1024, 7, ctypes.byref(h)) == binding.VBH_EINVAL
    p = binding.vbh_params(1000, 16, 16, 0.01, 0.04, 8, 6, 4.0, 4.0, 3.5, 2.5, 0.0, 1.0, 0)
    assert L.vbh_scene_create(ctypes.byref(p), ctypes.byref(h)) == binding.VBH_EINVAL
    p = binding.vbh_params(1024, 16, 16, 0.01, 0.005, 8, 6, 4.0, 4.0, 3.5, 2.5, 0.0, 1.0, 0)
    assert L.vbh_scene_create(ctypes.byref(p), ctypes.byref(h)) == binding.VBH_EINVAL
    assert L.vbh_insert(None, None, None, 0, None, None) == binding.VBH_EINVAL
    assert L.vbh_integrate_frame(None, None, None, None, 1, None) == binding.VBH_EINVAL
