"""Pins of two readings of the paper that no uniform input can tell apart.

- MC voxel colour (the paper sends one colour per MC voxel, Sec. 4.2; the reading taken here:
  the colour of the cell's corner-0 voxel).  Every voxel gets a colour of its own, so the
  expected colour of each surface cell is the hand-derived colour of its corner 0.
- The running mean at saturation (weight 1 per observation, W capped at 255, and then
  n = 256 observations in the mean).  After 255 equal observations t1 the mean is t1; each
  further observation t2 then moves it by 1/256 of the gap, so after k of them
  F = t2 + (t1 - t2) (255/256)^k (geometric closed form), and the colour follows the
  integer steps worked out by hand below.
Planted mistakes in the oracle's source ("colour from corner 6", "freeze at 255",
"n = 255 at saturation") each fail a pin.
"""
import numpy as np
import pytest

import oracle
from datagen.configs import Volume
from datagen.scenes import Camera
from oracle_variant import build_variant

VOL = Volume(slots=1 << 12, pool_blocks=1 << 12, voxel_size=0.01, trunc=0.04, depth_min=0.0,
             depth_max=float("inf"), log_capacity=1 << 16)
CAM8 = Camera(8, 6, 4.0, 4.0, 3.5, 2.5)
CAM2 = Camera(2, 2, 2.0, 2.0, 0.5, 0.5)
IDENT = np.hstack([np.eye(3), np.zeros((3, 1))])
OFFS = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)])


def voxels(keys):
    loc = np.arange(512)
    l = np.stack([loc % 8, (loc // 8) % 8, loc // 64], -1)
    return keys[:, None, :].astype(np.int64) * 8 + l[None]


def distinct_colour(g):
    """A colour that names its voxel: (8x + 1, 8y + 2, 8z + 3) for g in [0, 16)^3."""
    return np.stack([8 * g[..., 0] + 1, 8 * g[..., 1] + 2, 8 * g[..., 2] + 3], -1).astype(np.uint8)


def pin_mc_colour(L):
    keys = np.array([(x, y, z) for x in range(2) for y in range(2) for z in range(2)], np.int32)
    g = voxels(keys)
    # inside: below the plane z = 3.5 and beyond the plane x = 9.5 (voxel units)
    F = np.where((g[..., 2] < 3.5) | (g[..., 0] > 9.5), -0.3, 0.3).astype(np.float32)
    W = np.full(F.shape, 7, np.uint8)
    S = oracle.Scene(VOL, CAM8, L=L)
    assert S.write(keys, F, W, distinct_colour(g), 1) == 0
    mc, rgb = S.extract_mc(keys)
    checked = 0
    for b in range(keys.shape[0]):
        for l in range(512):
            c = g[b, l]
            if c.max() >= 15:  # the cell needs the +1 neighbour, beyond the 2^3 blocks
                assert mc[b, l] == 0
                continue
            inside = [(c + o)[2] < 3.5 or (c + o)[0] > 9.5 for o in OFFS]
            idx = sum(1 << k for k, i in enumerate(inside) if i)
            if idx in (0, 255):
                assert mc[b, l] == 0 and (rgb[b, l] == 0).all()
                continue
            assert mc[b, l] == idx
            # hand-derived: corner 0 of the cell at voxel c is c itself
            assert tuple(rgb[b, l]) == (8 * c[0] + 1, 8 * c[1] + 2, 8 * c[2] + 3), (c, rgb[b, l])
            checked += 1
    assert checked > 300


def observed_all(g, vs, mu, depths):
    """Voxels of the 2x2 identity camera observed in every frame of plane depths `depths`
    (float64 projection away from pixel-rounding ties)."""
    p = g * vs
    with np.errstate(divide="ignore", invalid="ignore"):
        u = CAM2.fx * (p[..., 0] / p[..., 2]) + CAM2.cx + 0.5
        v = CAM2.fy * (p[..., 1] / p[..., 2]) + CAM2.cy + 0.5
    ok = (np.abs(u - np.round(u)) > 1e-4) & (np.abs(v - np.round(v)) > 1e-4) & (p[..., 2] > 0)
    ok &= (u >= 0) & (u < CAM2.width) & (v >= 0) & (v < CAM2.height)
    for D in depths:
        ok &= (D - p[..., 2]) >= -mu + 1e-6
    return ok


# colour steps at saturation, c <- floor((255 c + c_obs + 128) / 256), worked by hand:
#   channel 0, from 40 towards 240: (255*40 + 368) / 256 = 10568 / 256 = 41.28 -> 41, then
#     42, 43, 44, 45 (remainders 71, 70, 69, 68)
#   channel 1, from 200 towards 10: (255*200 + 138) / 256 = 51138 / 256 = 199.76 -> 199,
#     then 198, 197, 196, 195
#   channel 2, 128 observed as 128: (255*128 + 256) / 256 = 128.5 -> 128
C1, C2 = (40, 200, 128), (240, 10, 128)
COLOUR_STEPS = [(41, 199, 128), (42, 198, 128), (43, 197, 128), (44, 196, 128), (45, 195, 128)]


def pin_saturation(L):
    D1, D2 = np.float32(0.2537), np.float32(0.2611)
    vs, mu = float(np.float32(0.01)), float(np.float32(0.04))
    S = oracle.Scene(VOL, CAM2, L=L)
    d1, d2 = np.full((2, 2), D1, np.float32), np.full((2, 2), D2, np.float32)
    c1 = np.broadcast_to(np.array(C1, np.uint8), (2, 2, 3)).copy()
    c2 = np.broadcast_to(np.array(C2, np.uint8), (2, 2, 3)).copy()
    for f in range(255):
        assert S.integrate(d1, c1, IDENT, f + 1) == 0
    keys = S.blocks()
    g = voxels(keys)
    sel = observed_all(g.astype(np.float64), vs, mu, [float(D1), float(D2)])
    assert sel.sum() > 100
    z = g[..., 2] * vs
    t1 = np.minimum(float(D1) - z, mu)
    t2 = np.minimum(float(D2) - z, mu)
    F, W, rgb, _ = S.read(keys)
    assert (W[sel] == 255).all() and np.abs(F[sel] - t1[sel]).max() < 1e-12
    assert (rgb[sel] == C1).all()
    moved = sel & (np.abs(t1 - t2) > 1e-3)
    assert moved.sum() > 50
    for k in range(1, 6):
        assert S.integrate(d2, c2, IDENT, 255 + k) == 0
        F, W, rgb, _ = S.read(keys)
        assert (W[sel] == 255).all()
        want = t2 + (t1 - t2) * (255.0 / 256.0) ** k
        assert np.abs(F[sel] - want[sel]).max() < 1e-12, f"saturated mean after {k} steps"
        assert (rgb[sel] == COLOUR_STEPS[k - 1]).all(), f"saturated colour after {k} steps"


def test_mc_colour_is_corner0_voxel():
    pin_mc_colour(oracle.lib())


def test_saturated_running_mean():
    pin_saturation(oracle.lib())


PLANTED = {
    "colour from corner 6": (pin_mc_colour, "const int kc = 0;", "const int kc = 6;"),
    "freeze at 255": (pin_saturation, "const int w_old = b.W[l];",
                      "const int w_old = b.W[l];\n        if (w_old == 255) continue;"),
    "n = 255 at saturation": (pin_saturation, "const int n = w_old + 1;", "const int n = std::min(w_old + 1, 255);"),
}


@pytest.mark.parametrize("name", sorted(PLANTED))
def test_planted_reading_mistakes_are_caught(name):
    pin, old, new = PLANTED[name]
    L = build_variant("oracle.cpp", old, new)
    with pytest.raises(AssertionError):
        pin(L)
