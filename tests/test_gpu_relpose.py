"""GPU parity of the relative-pose pieces (Sec. III-D) against the FP64
oracle: the unprojection with nearest-neighbour scales (oracle/relpose.py),
the confidence-masked L1 of Eq. (20)-(21) (oracle.masked_l1), and an
end-to-end relative pose between two room frames.

Tolerances: means are FP32 evaluations of (x + 1/2 - cx) / fx * z, relative
error <= 1e-6; a log scale is the log of a mean of three FP32 distances
(relative error ~1e-7), and a near-tie between neighbours changes the mean
by no more than the tie's gap, so |d log s| <= 1e-5; the masked L1's
gradient is a sign under a mask both sides decide identically (bit-exact),
its loss a sum of FP32 differences (relative 1e-6)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import relpose as ORP
from paper_2410_08743_amd import relpose as RP
from paper_2410_08743_amd import render as R
from paper_2410_08743_amd import synthetic as S

from parity_util import random_case

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("stride,roi", [(3, (16, 16, 70, 45)), (1, None), (5, (0, 32, 96, 40))])
def test_unproject_matches_oracle(stride, roi):
    rng = np.random.default_rng(stride)
    cam = S.Camera(96, 80, 70.3, 71.1, 47.6, 39.2, roi=roi)
    w, h = (roi[2], roi[3]) if roi else (96, 80)
    depth = rng.uniform(0.8, 6.0, (h, w)).astype(np.float32)
    depth[rng.random((h, w)) < 0.03] = 0.0
    depth[0, 0] = np.nan
    image = rng.uniform(0, 1, (3, h, w)).astype(np.float32)
    raw = RP.unproject(cam, torch.tensor(depth, device=DEV), torch.tensor(image, device=DEV),
                       stride, opacity=0.1, sh_degree=1)
    ref = ORP.unproject(depth, image, cam, stride, opacity=0.1)
    got_m = raw.means.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got_m - ref["means"]) / np.maximum(1.0, np.abs(ref["means"]))) <= 1e-6
    assert np.max(np.abs(raw.log_scales.cpu().numpy() - ref["log_scales"])) <= 1e-5
    assert np.array_equal(raw.quats.cpu().numpy(), ref["quats"].astype(np.float32))
    assert np.max(np.abs(raw.logit_opacities.cpu().numpy() - ref["logit_opacities"])) <= 1e-6
    sh = raw.sh.cpu().numpy()
    assert np.max(np.abs(sh[:, :1, :] - ref["sh"])) <= 1e-6
    assert np.array_equal(sh[:, 1:, :], np.zeros_like(sh[:, 1:, :]))


def test_masked_l1_matches_oracle():
    sc, cam, pose = random_case(41, 1, 90, 70, 3000)
    g = R.GaussianParams.from_set(sc, DEV)
    rast = R.Rasterizer(0)
    img, alpha = rast.forward(g, [cam], torch.tensor(pose[None], device=DEV), alphas=True)
    target = torch.tensor(np.random.default_rng(42).uniform(0, 1, img.numel()).astype(np.float32),
                          device=DEV)
    loss, grad = R.masked_l1([cam], img, target, alpha)
    a = alpha.cpu().numpy().astype(np.float64)
    mask = a > 0.99
    assert 0.05 < mask.mean() < 0.95          # both sides of the threshold occur
    ref_val, ref_grad = oracle.masked_l1(img.cpu().numpy().reshape(3, 70, 90),
                                         target.cpu().numpy().reshape(3, 70, 90),
                                         (1.0 - a).reshape(70, 90))
    assert np.array_equal(grad.cpu().numpy().reshape(3, 70, 90), ref_grad.astype(np.float32))
    assert abs(loss.item() - ref_val) <= 1e-6 * ref_val


def test_masked_l1_views_are_independent():
    cams, imgs, tgts, alphas = [], [], [], []
    for k, (W, H) in enumerate(((64, 48), (90, 70))):
        sc, cam, pose = random_case(50 + k, 0, W, H, 2000)
        g = R.GaussianParams.from_set(sc, DEV)
        im, al = R.Rasterizer(0).forward(g, [cam], torch.tensor(pose[None], device=DEV), alphas=True)
        cams.append(cam)
        imgs.append(im)
        alphas.append(al)
        tgts.append(torch.rand_like(im))
    loss, grads = R.masked_l1(cams, imgs, tgts, alphas)
    for k in range(2):
        lk, gk = R.masked_l1([cams[k]], imgs[k], tgts[k], alphas[k])
        assert torch.equal(loss[k:k + 1], lk) and torch.equal(grads[k], gk)


def test_relative_pose_between_room_frames():
    """Consecutive frames 60 and 61 of the room trajectory (a clear view of
    the room), frame 60's depth map from the expected-depth render of the
    scene; the solve at the settings of Sec. IV (200 masked-L1 steps,
    1e-3 -> 1e-4)."""
    wl = S.room(n=150_000, n_frames=63)
    cam = S.Camera(320, 180, 160.0, 160.0, 160.0, 90.0)
    g = R.GaussianParams.from_set(wl.scene, DEV)
    traj = wl.extra["trajectory"]
    P0, P1 = traj[60].astype(np.float64), traj[61].astype(np.float64)
    rast = R.Rasterizer(0)
    t0 = torch.tensor(P0[None].astype(np.float32), device=DEV)
    i0, _ = rast.forward(g, [cam], t0)
    i0 = i0.clone().view(3, 180, 320)
    i1, _ = rast.forward(g, [cam], torch.tensor(P1[None].astype(np.float32), device=DEV))
    i1 = i1.clone()
    gz = R.GaussianParams.from_set(S.depth_coloured(wl.scene, P0), DEV)
    dimg, al = R.Rasterizer(0).forward(gz, [cam], t0, alphas=True)
    depth = (dimg.view(3, 180, 320)[0] / al.view(180, 320).clamp_min(1e-6)).contiguous()
    rel, raw = RP.relative_pose(cam, i0, depth, i1, stride=2)
    # ground truth: frame t+1's world->camera composed with frame t's camera->world
    H0 = np.vstack([P0, [0, 0, 0, 1]])
    H1 = np.vstack([P1, [0, 0, 0, 1]])
    gt = (H1 @ np.linalg.inv(H0))[:3]
    ident = np.hstack([np.eye(3), np.zeros((3, 1))])
    e_start = S.pose_error(ident, gt)
    e_end = S.pose_error(rel.cpu().numpy(), gt)
    assert e_end[0] < 0.05 * e_start[0] and e_end[1] < 0.1 * e_start[1], (e_start, e_end)
