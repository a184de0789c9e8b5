"""MI355X (gfx950) voxel-block-hashing hot path of SLAMCast (Stotko et al., TVCG 2019).

The compute path is libvbh.so (hand-written HIP kernels behind the C ABI in
include/vbh.h); this package only marshals torch tensors into it.
"""
from .binding import (ChainedMap, Map, Scene, Server, VbhError, lib, make_params, vbh_params, vbh_stats,  # noqa: F401
                      exported_names, vbh_mc_triangulate, VBH_ABSENT, VBH_OP_INSERT, VBH_OP_FIND, VBH_OP_ERASE,
                      VBH_HASH_SPATIAL, VBH_HASH_MIX64)
