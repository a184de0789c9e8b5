"""Pins of the oracle's differentiable form: analytic float64 gradient against central
finite differences of the frozen loss (h = 1e-4), a hand-derived closed form, and a
directional derivative over all inputs."""
import numpy as np
import pytest

from datagen import configs
from datagen.configs import Volume
from datagen.scenes import Camera, look_at

VOL = Volume(slots=1 << 14, pool_blocks=1 << 14, voxel_size=0.02, trunc=0.08, depth_min=0.0,
             depth_max=float("inf"), log_capacity=1 << 16)


def small_problem(n_frames=3, n_samples=300, seed=0):
    cam = Camera(48, 36, 40.0, 40.0, 23.5, 17.5)
    scene = configs.box_room_scene(1805, VOL.voxel_size)
    from datagen.scenes import render_frames
    poses = np.stack([look_at([0.8 * np.cos(a), 0.8 * np.sin(a), 0.05], [0, 0, 0]) for a in
                      np.linspace(0.0, 0.5, n_frames)])
    depth, _ = render_frames(scene, cam, poses)
    depth = depth.numpy()
    rng = np.random.default_rng(seed)
    valid = np.flatnonzero(depth.reshape(-1) > 0)
    pick = np.sort(rng.choice(valid, n_samples, replace=False))
    hw = cam.width * cam.height
    return cam, depth, poses, (pick // hw).astype(np.int32), (pick % hw).astype(np.int32)


@pytest.fixture(scope="module")
def prob(orc):
    cam, depth, poses, sf, sp = small_problem()
    return orc.Diff(VOL, cam, depth, poses, sf, sp), depth


def test_problem_is_nontrivial(prob):
    D, _ = prob
    info = D.info()
    assert info["kept"] > 100 and info["grad_voxels"] > 500
    assert D.loss() > 0


def test_pose_gradient_matches_fd(orc, prob):
    D, _ = prob
    gD, gxi = D.grad()
    fd = np.array([[D.fd_pose(f, a) for a in range(6)] for f in range(D.F)])
    err = orc.rel_err(gxi, fd)
    assert err.max() < 1e-4, (err.max(), gxi, fd)
    assert np.abs(fd).max() > 1e-3


def test_three_point_fd_converges_at_second_order(orc, prob):
    """The plain central difference approaches the analytic gradient as h^2."""
    D, _ = prob
    _, gxi = D.grad()
    for f, a in [(0, 0), (0, 5), (2, 5), (1, 3)]:
        e3 = abs(D.fd_pose(f, a, 1e-3, points=3) - gxi[f, a])
        e4 = abs(D.fd_pose(f, a, 1e-4, points=3) - gxi[f, a])
        assert e4 < 0.02 * e3 + 1e-12, (f, a, e3, e4)


def test_depth_gradient_matches_fd(orc, prob):
    D, depth = prob
    gD, _ = D.grad()
    rng = np.random.default_rng(1)
    # pixels carrying samples, and pixels that feed voxels with nonzero dL/dF
    cand = [(int(f), int(p)) for f, p in zip(D.sf[:20], D.sp[:20])]
    nz = np.argwhere(gD != 0)
    nz = nz[rng.choice(len(nz), 30, replace=False)]
    cand += [(int(f), int(p)) for f, p in nz]
    g = np.array([gD[f, p] for f, p in cand])
    fd = np.array([D.fd_depth(f, p) for f, p in cand])
    err = orc.rel_err(g, fd, scale_ref=np.abs(gD).max())
    assert err.max() < 1e-4, err.max()


def test_directional_derivative(orc, prob):
    D, depth = prob
    gD, gxi = D.grad()
    rng = np.random.default_rng(2)
    vD = rng.standard_normal(gD.shape) * (depth.reshape(D.F, -1) > 0)
    vx = rng.standard_normal(gxi.shape)
    fd = D.fd_direction(vD, vx)
    an = float((gD * vD).sum() + (gxi * vx).sum())
    assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-12) + 1e-12


def test_closed_form_two_planes(orc):
    """Two identity-pose frames seeing fronto-parallel planes at D1 and D2 and one sample on
    the optical axis of frame 1: F_tri = (D2 - D1)/2, and
    dL/dD1 = -(D2-D1)/2, dL/dD2 = (D2-D1)/2, dL/drho1_z = -(D2-D1)/2, dL/drho2_z = (D2-D1)/2."""
    cam = Camera(7, 5, 4.0, 4.0, 3.0, 2.0)
    D1, D2 = 1.0037, 1.0213
    depth = np.stack([np.full((5, 7), D1, np.float32), np.full((5, 7), D2, np.float32)])
    ident = np.hstack([np.eye(3), np.zeros((3, 1))])
    pix = 2 * 7 + 3  # (u, v) = (cx, cy): the optical axis
    D = orc.Diff(VOL, cam, depth, [ident, ident], np.array([0], np.int32), np.array([pix], np.int32))
    d1, d2 = float(np.float32(D1)), float(np.float32(D2))
    assert D.info()["kept"] == 1
    assert abs(D.info()["f_samples"][0] - (d2 - d1) / 2) < 1e-12
    gD, gxi = D.grad()
    h = (d2 - d1) / 2
    assert abs(gD[0, pix] + h) < 1e-12 and abs(gD[1, pix] - h) < 1e-12
    assert np.abs(np.delete(gD.reshape(-1), [pix, 35 + pix])).max() < 1e-12
    assert abs(gxi[0, 2] + h) < 1e-12 and abs(gxi[1, 2] - h) < 1e-12
    assert np.abs(np.delete(gxi.reshape(-1), [2, 8])).max() < 1e-12


XI_REF = np.array([[0.03, -0.02, 0.01, 0.05, -0.04, 0.08],
                   [-0.02, 0.015, 0.03, -0.06, 0.02, 0.07],
                   [0.01, 0.02, -0.025, 0.04, 0.09, -0.05]])


def test_gradient_at_nonzero_xi_matches_fd(orc):
    """At a nonzero reference xi (poses Exp(xi) T0, tens of mrad and cm), the analytic
    gradient - the left-perturbation gradient mapped through J_l(xi)^T - equals 5-point
    central differences of L(Exp(xi + h e) T0) in every pose coordinate and in sampled
    depths; without the Jacobian the pose gradient is off by far more than the bar."""
    cam, depth, poses, sf, sp = small_problem()
    D = orc.Diff(VOL, cam, depth, poses, sf, sp, xi_ref=XI_REF)
    assert D.info()["kept"] > 100
    gD, gxi = D.grad()
    fd = np.array([[D.fd_pose(f, a) for a in range(6)] for f in range(D.F)])
    err = orc.rel_err(gxi, fd)
    assert err.max() < 1e-4, (err.max(), gxi, fd)
    rng = np.random.default_rng(3)
    nz = np.argwhere(gD != 0)
    pick = nz[rng.choice(len(nz), 24, replace=False)]
    fdp = np.array([D.fd_depth(int(f), int(p)) for f, p in pick])
    e = orc.rel_err(np.array([gD[f, p] for f, p in pick]), fdp, scale_ref=np.abs(gD).max())
    assert e.max() < 1e-4
    # the plain left-perturbation gradient at the same poses is a different vector
    J = np.stack([left_jacobian_closed(XI_REF[f]) for f in range(D.F)])
    g_left = np.linalg.solve(np.transpose(J, (0, 2, 1)), gxi[..., None])[..., 0]
    assert orc.rel_err(g_left, fd).max() > 1e-2


def left_jacobian_closed(xi):
    """Closed form of the SE(3) left Jacobian, [[J, Q], [0, J]] (Barfoot and Furgale 2014),
    written independently of the oracle's series; used to undo it above."""
    rho, phi = xi[:3], xi[3:]
    t = np.linalg.norm(phi)

    def hat(w):
        return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    P, R = hat(phi), hat(rho)
    J = np.eye(3) + (1 - np.cos(t)) / t ** 2 * P + (t - np.sin(t)) / t ** 3 * P @ P
    Q = (0.5 * R + (t - np.sin(t)) / t ** 3 * (P @ R + R @ P + P @ R @ P)
         + (t ** 2 + 2 * np.cos(t) - 2) / (2 * t ** 4) * (P @ P @ R + R @ P @ P - 3 * P @ R @ P)
         + (2 * t - 3 * np.sin(t) + t * np.cos(t)) / (2 * t ** 5) * (P @ R @ P @ P + P @ P @ R @ P))
    out = np.zeros((6, 6))
    out[:3, :3], out[:3, 3:], out[3:, 3:] = J, Q, J
    return out


def test_left_jacobian_closed_form_against_fd_of_exp(orc):
    """The closed form used above satisfies Exp(xi + d) ~ Exp(J d) Exp(xi): checked by
    central differences of the matrix exponential of the 4x4 twist (scipy's expm)."""
    from scipy.linalg import expm, logm

    def twist(x):
        T = np.zeros((4, 4))
        T[:3, :3] = np.array([[0, -x[5], x[4]], [x[5], 0, -x[3]], [-x[4], x[3], 0]])
        T[:3, 3] = x[:3]
        return T

    for xi in XI_REF:
        E = expm(twist(xi))
        J = left_jacobian_closed(xi)
        h = 1e-6
        for a in range(6):
            e = np.zeros(6)
            e[a] = h
            D = (expm(twist(xi + e)) - expm(twist(xi - e))) @ np.linalg.inv(E) / (2 * h)
            v = np.array([D[0, 3], D[1, 3], D[2, 3], D[2, 1], D[0, 2], D[1, 0]])
            assert np.abs(v - J[:, a]).max() < 1e-7
        assert np.allclose(logm(E).real, twist(xi), atol=1e-12)
