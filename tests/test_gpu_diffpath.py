"""Differentiation path: the torch.autograd.Function over the library on
sub-crops of the tracking workload (the 500k-Gaussian room, 1200x680).
Gradients of every parameter group and of the pose twist are checked against
the FP64 oracle's backward on 16-aligned 64x64 regions along the
trajectory, and the oracle's pose gradient against its own central
differences on the same regions of a smaller room (the difference checks
need every discrete decision of the render to stay fixed, which a
500k-Gaussian crop rarely allows at FP64-resolvable steps)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_08743_amd import render as R
from paper_2410_08743_amd import synthetic as S
from tests.parity_util import assert_grad_close, f32_camera
from tests.test_oracle_gradients import _fd_pose, _loss

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (frame, roi x, roi y): eight 64x64 regions along the trajectory
CROPS = [(0, 560, 304), (13, 96, 160), (27, 1024, 480), (40, 304, 48),
         (54, 768, 592), (67, 640, 336), (81, 16, 400), (95, 912, 128)]


@pytest.fixture(scope="module")
def room():
    return S.room()


def _autograd_grads(g, cam, pose, W):
    params = [t.clone().requires_grad_(True) for t in (g.means, g.scales, g.quats, g.opacities, g.sh)]
    tau = torch.zeros((1, 6), device=DEV, requires_grad=True)
    img = R.render(g, [cam], torch.tensor(pose[None], device=DEV), tau=tau, params=params)
    (img * torch.tensor(W.ravel(), device=DEV)).sum().backward()
    names = ("means", "scales", "quats", "opacities", "sh")
    out = {k: p.grad.cpu().numpy() for k, p in zip(names, params)}
    out["pose"] = tau.grad.cpu().numpy()[0]
    return out


def test_autograd_crops_match_the_oracle(room):
    g = R.GaussianParams.from_set(room.scene, DEV)
    traj = room.extra["trajectory"]
    for k, (frame, x, y) in enumerate(CROPS):
        cam = f32_camera(room.camera.with_roi((x, y, 64, 64)))
        W = S.upstream(700 + k, (3, 64, 64))
        got = _autograd_grads(g, cam, traj[frame], W)
        ref = oracle.backward(room.scene, cam, traj[frame], W)
        print(f"crop {k}: frame {frame} roi ({x}, {y})", flush=True)
        for name in ("means", "scales", "quats", "opacities", "sh"):
            assert_grad_close(got[name], ref[name], f"crop {k} {name}")
        assert_grad_close(got["pose"][:3], ref["pose"][:3], f"crop {k} rho")
        assert_grad_close(got["pose"][3:], ref["pose"][3:], f"crop {k} phi")


def test_pose_gradient_of_crops_by_central_differences():
    small = S.room(n=20_000, n_frames=100)
    g = R.GaussianParams.from_set(small.scene, DEV)
    traj = small.extra["trajectory"]
    sc64 = S.GaussianSet(*(np.asarray(a, np.float64) for a in
                           (small.scene.means, small.scene.scales, small.scene.quats,
                            small.scene.opacities, small.scene.sh)), 3)
    checked = 0
    for k, (frame, x, y) in enumerate(CROPS):
        cam = f32_camera(small.camera.with_roi((x, y, 64, 64)))
        pose = traj[frame].astype(np.float64)
        W = S.upstream(800 + k, (3, 64, 64))
        _, sig0 = _loss(sc64, cam, pose, W)
        fd = _fd_pose(sc64, cam, pose, W, sig0)
        an = oracle.backward(sc64, cam, pose, W)["pose"]
        got = _autograd_grads(g, cam, traj[frame], W)["pose"]
        ok = np.isfinite(fd)
        if ok.sum() < 5:
            continue
        scale = max(np.linalg.norm(an[ok]), 1e-12)
        assert np.linalg.norm(an[ok] - fd[ok]) / scale < 1e-5, (k, an, fd)
        assert_grad_close(got[:3], an[:3], f"crop {k} rho")
        assert_grad_close(got[3:], an[3:], f"crop {k} phi")
        checked += 1
    assert checked >= 6


def test_full_frame_matches_the_oracle(room):
    """A whole 1200x680 frame of the tracking workload (the size the
    tracking benchmark renders): image and pose gradient of the L1 loss's
    upstream gradient against the oracle."""
    g = R.GaussianParams.from_set(room.scene, DEV)
    cam = f32_camera(room.camera)
    pose = room.extra["trajectory"][60]
    rast = R.Rasterizer(0)
    img, _ = rast.forward(g, [cam], torch.tensor(pose[None], device=DEV))
    ref = oracle.render(room.scene, cam, pose)
    got = img.cpu().numpy().reshape(3, cam.height, cam.width)
    strad = ref["straddle"]
    err = np.abs(got - ref["image"]).max(axis=0)
    assert strad.mean() <= 2e-3 and float(err[~strad].max()) <= 1e-4
    W = S.upstream(760, (3, cam.height, cam.width))
    gr = rast.backward(g, [cam], torch.tensor(pose[None], device=DEV),
                       torch.tensor(W.ravel(), device=DEV), want=())
    back = oracle.backward(room.scene, cam, pose, W)
    gp = gr["pose"][0].cpu().numpy()
    assert_grad_close(gp[:3], back["pose"][:3], "rho")
    assert_grad_close(gp[3:], back["pose"][3:], "phi")
