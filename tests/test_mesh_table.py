"""The library's triangulation table (host query vbh_mc_case, no GPU needed) against the
oracle's triangulation of every case, triangle by triangle."""
import ctypes as C

import numpy as np

EDGES = [(0, 1), (1, 2), (2, 3), (3, 0), (4, 5), (5, 6), (6, 7), (7, 4), (0, 4), (1, 5), (2, 6), (3, 7)]
CORNERS = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)])


def test_every_case_matches_the_oracle(orc):
    from paper_1805_03709_amd import binding
    L = binding.lib()
    mid = {tuple(CORNERS[a] + CORNERS[b]): e for e, (a, b) in enumerate(EDGES)}  # doubled midpoints
    keys = np.zeros((1, 3), np.int32)
    total = 0
    for idx in range(256):
        buf = (C.c_int8 * 15)()
        nt = L.vbh_mc_case(idx, buf)
        got = [tuple(buf[3 * t:3 * t + 3]) for t in range(nt)]
        assert all(v == -1 for v in buf[3 * nt:])
        mcv = np.zeros((1, 512), np.uint32)
        mcv[0, 0] = idx
        pos, _ = orc.mc_triangles(keys, mcv, 2.0)  # voxel 2: positions are the doubled midpoints
        want = [tuple(mid[tuple(int(round(x)) for x in v)] for v in tri) for tri in pos]
        assert got == want, idx
        total += nt
    assert L.vbh_mc_case(256, None) < 0 and L.vbh_mc_case(-1, None) < 0
    assert total > 256
