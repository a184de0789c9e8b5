"""GPU parity of the differentiable form against the float64 oracle: loss and sampled F,
and the gradients w.r.t. every pixel depth and every pose coordinate (analytic oracle
gradient everywhere, 5-point central differences at h = 1e-4 on a seeded subset).
Bar: 1e-4 relative, denominator max(|g_ref|, 1e-3 max|g_ref|)."""
import numpy as np
import pytest
import torch

from datagen import configs
from gpu_util import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-4


def run_gpu(vbh, vol, cam, depth, poses, sf, sp, xi=None):
    from paper_1805_03709_amd.autograd import DiffFusion
    E = DiffFusion(vbh.make_params(vol, cam), depth.shape[0])
    d, f, p = to_dev(depth), to_dev(sf), to_dev(sp)
    x = None if xi is None else to_dev(np.asarray(xi, np.float32))
    loss, fs = E.vbh_diff_forward(d, poses, f, p, xi=x)
    gD, gxi = E.vbh_diff_backward(d, poses, f, p, torch.ones((), device="cuda"), xi=x)
    return E, float(loss.cpu()), fs.cpu().numpy(), gD.cpu().numpy().reshape(depth.shape[0], -1), gxi.cpu().numpy()


def check(orc, O, loss, fs, gD, gxi, n_fd_pix=64, fd_pose=True):
    info = O.info()
    of = info["f_samples"]
    assert np.array_equal(np.isnan(fs), np.isnan(of)), "sample masks differ"
    m = ~np.isnan(of)
    say(f"  kept {m.sum()} / {of.size} samples, {info['grad_voxels']} corner voxels, "
        f"max|F_gpu-F64| {np.abs(fs[m] - of[m]).max():.3g}")
    assert np.abs(fs[m] - of[m]).max() < 1e-5
    oloss = O.loss()
    assert abs(loss - oloss) <= 1e-5 * oloss
    ogD, ogxi = O.grad()
    e_xi = orc.rel_err(gxi, ogxi)
    e_d = orc.rel_err(gD, ogD)
    say(f"  loss {loss:.6g} vs {oloss:.6g}; max rel err: xi {e_xi.max():.3g}, depth {e_d.max():.3g}")
    assert e_xi.max() < TOL and e_d.max() < TOL
    if fd_pose:
        fd = np.array([[O.fd_pose(f, a) for a in range(6)] for f in range(O.F)])
        e = orc.rel_err(gxi, fd)
        say(f"  pose vs 5-point FD: max rel err {e.max():.3g}")
        assert e.max() < TOL
    rng = np.random.default_rng(7)
    nz = np.argwhere(ogD != 0)
    pick = nz[rng.choice(len(nz), min(n_fd_pix, len(nz)), replace=False)]
    fdp = np.array([O.fd_depth(int(f), int(p)) for f, p in pick])
    e = orc.rel_err(np.array([gD[f, p] for f, p in pick]), fdp, scale_ref=np.abs(ogD).max())
    say(f"  depth vs 5-point FD ({len(pick)} pixels): max rel err {e.max():.3g}")
    assert e.max() < TOL


def test_small_problem(orc):
    vbh = require_gpu()
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_diff import VOL, small_problem
    cam, depth, poses, sf, sp = small_problem()
    say("[diff small]")
    E, loss, fs, gD, gxi = run_gpu(vbh, VOL, cam, depth, poses, sf, sp)
    O = orc.Diff(VOL, cam, depth, poses, sf, sp)
    check(orc, O, loss, fs, gD, gxi)


def test_full_size_sixteen_frames(orc):
    """Frames 500-515 of the 640x480 sequence, 2 cm voxels, 8 cm truncation, 100k samples."""
    vbh = require_gpu()
    say("[diff full] generating")
    _, depth, _, poses, sf, sp = configs.diff_inputs(device="cuda")
    depth = depth.cpu().numpy()
    E, loss, fs, gD, gxi = run_gpu(vbh, configs.DIFF_VOL, configs.FULL_CAM, depth, poses, sf, sp)
    say("[diff full] oracle")
    O = orc.Diff(configs.DIFF_VOL, configs.FULL_CAM, depth, poses, sf, sp)
    check(orc, O, loss, fs, gD, gxi, n_fd_pix=48)


def test_autograd_function_matches_abi():
    vbh = require_gpu()
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_diff import VOL, small_problem
    from paper_1805_03709_amd.autograd import DiffFusion, TSDFSampleLoss
    cam, depth, poses, sf, sp = small_problem()
    E = DiffFusion(vbh.make_params(VOL, cam), depth.shape[0])
    d = to_dev(depth).requires_grad_(True)
    xi = torch.zeros((depth.shape[0], 6), device="cuda", requires_grad=True)
    f, p = to_dev(sf), to_dev(sp)
    loss = TSDFSampleLoss.apply(d, xi, E, poses, f, p)
    (3.0 * loss).backward()
    E2 = DiffFusion(vbh.make_params(VOL, cam), depth.shape[0])
    l2, _ = E2.vbh_diff_forward(d.detach(), poses, f, p)
    gD, gxi = E2.vbh_diff_backward(d.detach(), poses, f, p, torch.full((), 3.0, device="cuda"))
    assert abs(float(loss.detach()) - float(l2)) <= 1e-6 * float(l2)
    assert torch.allclose(d.grad, gD, rtol=1e-5, atol=1e-9)
    assert torch.allclose(xi.grad, gxi, rtol=1e-5, atol=1e-9)


def test_nonzero_xi_against_oracle(orc):
    """Poses Exp(xi) T0 at a nonzero xi: the library composes them, and its dL/dxi (left
    gradient through J_l(xi)^T) matches the oracle's analytic gradient at that reference
    point and 5-point differences of L(Exp(xi + h e) T0); the autograd function returns
    the same gradients as the ABI."""
    vbh = require_gpu()
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_diff import VOL, XI_REF, small_problem
    from paper_1805_03709_amd.autograd import DiffFusion, TSDFSampleLoss
    cam, depth, poses, sf, sp = small_problem()
    xi32 = XI_REF.astype(np.float32)
    say("[diff nonzero xi]")
    E, loss, fs, gD, gxi = run_gpu(vbh, VOL, cam, depth, poses, sf, sp, xi=xi32)
    O = orc.Diff(VOL, cam, depth, poses, sf, sp, xi_ref=xi32.astype(np.float64))
    check(orc, O, loss, fs, gD, gxi)
    # through autograd
    E2 = DiffFusion(vbh.make_params(VOL, cam), depth.shape[0])
    d = to_dev(depth).requires_grad_(True)
    xi = to_dev(xi32).requires_grad_(True)
    l2 = TSDFSampleLoss.apply(d, xi, E2, poses, to_dev(sf), to_dev(sp))
    l2.backward()
    assert abs(float(l2.detach()) - loss) <= 1e-6 * loss
    assert np.allclose(xi.grad.cpu().numpy(), gxi, rtol=1e-5, atol=1e-9)
    assert np.allclose(d.grad.cpu().numpy().reshape(gD.shape), gD, rtol=1e-5, atol=1e-9)
    # the backward refuses inputs other than the forward's
    with pytest.raises(vbh.VbhError):
        E.vbh_diff_backward(to_dev(depth), poses, to_dev(sf), to_dev(sp), torch.ones((), device="cuda"))
