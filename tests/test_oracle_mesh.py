"""Pins of the oracle's client triangulation (Sec. 4.3; vertices without interpolation): on
MC voxels built directly from analytic surfaces, the mesh is closed, consistently
oriented with outward normals, has the Euler characteristic of the surface's genus,
encloses the right volume, and every vertex is the midpoint of a sign-changing lattice
edge within half a voxel of the true surface.  Single-corner cases are checked by hand."""
import numpy as np
import pytest

CORNERS = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)])


def mc_blocks(sdf, lo, hi, vs):
    """MC voxels (index | RGB << 8) of every block touching the lattice box [lo, hi) (in
    voxels): bit k of a cell's index is set iff the SDF is negative at corner k.  The
    colour encodes the cell's x, y, z modulo 256 so that it can be checked."""
    B0, B1 = np.floor_divide(lo, 8), np.floor_divide(hi - 1, 8)
    keys, mcv = [], []
    loc = np.arange(512)
    l3 = np.stack([loc % 8, (loc // 8) % 8, loc // 64], -1)
    for bx in range(B0[0], B1[0] + 1):
        for by in range(B0[1], B1[1] + 1):
            for bz in range(B0[2], B1[2] + 1):
                g = np.array([bx, by, bz]) * 8 + l3
                idx = np.zeros(512, np.uint32)
                for k in range(8):
                    p = (g + CORNERS[k]).astype(np.float64) * vs
                    idx |= (sdf(p) < 0).astype(np.uint32) << k
                rgb = (g % 256).astype(np.uint32)
                v = np.where((idx == 0) | (idx == 255), 0, idx | rgb[:, 0] << 8 | rgb[:, 1] << 16 | rgb[:, 2] << 24)
                keys.append((bx, by, bz))
                mcv.append(v.astype(np.uint32))
    return np.array(keys, np.int32), np.stack(mcv)


def mesh_checks(pos, vs, sdf):
    q = np.round(pos / (0.5 * vs)).astype(np.int64)  # half-voxel units, exact
    assert np.array_equal(q * np.float32(0.5 * vs), pos.astype(np.float64)) or np.allclose(q * 0.5 * vs, pos, atol=1e-6)
    # every vertex is the midpoint of a lattice edge (exactly one odd coordinate) whose
    # ends have opposite SDF signs
    v = q.reshape(-1, 3)
    odd = v % 2
    assert (odd.sum(1) == 1).all()
    a = (v - odd) // 2
    b = (v + odd) // 2
    sa, sb = sdf(a * vs) < 0, sdf(b * vs) < 0
    assert (sa != sb).all()
    # closed and consistently oriented: every directed edge once, its reverse once
    tri = [tuple(map(tuple, t)) for t in q]
    directed = {}
    for t in tri:
        for i in range(3):
            e = (t[i], t[(i + 1) % 3])
            directed[e] = directed.get(e, 0) + 1
    assert all(c == 1 for c in directed.values())
    assert all((e[1], e[0]) in directed for e in directed)
    V = len({p for t in tri for p in t})
    E = len(directed) // 2
    F = len(tri)
    vol = np.einsum("ij,ij->i", pos[:, 0].astype(np.float64),
                    np.cross(pos[:, 1].astype(np.float64), pos[:, 2].astype(np.float64))).sum() / 6
    return V - E + F, vol


def test_sphere_closed_oriented_genus0_and_volume(orc):
    vs, r, c = 0.01, 0.1037, np.array([0.0031, -0.0017, 0.0043])
    sdf = lambda p: np.linalg.norm(p - c, axis=-1) - r
    keys, mcv = mc_blocks(sdf, np.array([-14, -14, -14]), np.array([14, 14, 14]), vs)
    pos, rgb = orc.mc_triangles(keys, mcv, vs)
    assert pos.shape[0] > 1000
    chi, vol = mesh_checks(pos, vs, sdf)
    assert chi == 2
    assert abs(vol / (4 / 3 * np.pi * r ** 3) - 1) < 0.02
    # every vertex within half a voxel of the sphere
    d = np.abs(np.linalg.norm(pos.reshape(-1, 3).astype(np.float64) - c, axis=-1) - r)
    assert d.max() <= 0.5 * vs + 1e-6


def test_torus_has_genus_one(orc):
    vs, R, r = 0.01, 0.0813, 0.0347
    def sdf(p):
        q = np.stack([np.hypot(p[..., 0], p[..., 1]) - R, p[..., 2]], -1)
        return np.linalg.norm(q, axis=-1) - r
    keys, mcv = mc_blocks(sdf, np.array([-13, -13, -6]), np.array([13, 13, 6]), vs)
    pos, _ = orc.mc_triangles(keys, mcv, vs)
    chi, vol = mesh_checks(pos, vs, sdf)
    assert chi == 0
    assert abs(vol / (2 * np.pi ** 2 * R * r ** 2) - 1) < 0.05


def test_single_corner_cases_and_cut_off(orc):
    keys = np.zeros((1, 3), np.int32)
    for idx in (0, 255):
        mcv = np.zeros((1, 512), np.uint32)
        mcv[0, 0] = idx | 0xABCDEF00
        assert orc.mc_triangles(keys, mcv, 1.0)[0].shape[0] == 0
    for k in range(8):
        for inside_only in (True, False):
            idx = (1 << k) if inside_only else 255 ^ (1 << k)
            mcv = np.zeros((1, 512), np.uint32)
            mcv[0, 9] = idx | (7 << 8) | (8 << 16) | (9 << 24)  # cell at local (1, 1, 0)
            pos, rgb = orc.mc_triangles(keys, mcv, 1.0)
            assert pos.shape[0] == 1 and tuple(rgb[0]) == (7, 8, 9)
            corner = np.array([1, 1, 0]) + CORNERS[k]
            # the three vertices are the midpoints of the corner's three edges
            d = pos[0] - corner
            assert np.allclose(np.sort(np.abs(d), axis=1), [[0, 0, 0.5]] * 3)
            n = np.cross(pos[0][1] - pos[0][0], pos[0][2] - pos[0][0])
            away = pos[0].mean(0) - corner
            # normals point from inside to outside: away from an inside corner, towards an outside one
            assert (n @ away > 0) == inside_only
