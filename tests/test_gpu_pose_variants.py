"""GPU checks of the pose variants: the T x SO(3) Adam step against its
oracle (oracle/pose_variants.py), solves in both parametrisations, and the
multi-hypothesis solve (several starting poses of one image as the views of
one launch).  The T x SO(3) step runs in FP64 on FP32 poses, so a step
agrees with the oracle to FP32 rounding of the pose entries (2e-6)."""
import numpy as np
import pytest
import torch

from oracle import pose_variants as PV
from paper_2410_08743_amd import render as R
from paper_2410_08743_amd import synthetic as S

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_txso3_adam_kernel_matches_oracle():
    rng = np.random.default_rng(5)
    V, K = 4, 6
    poses = np.stack([S.random_pose_near_identity(60 + k, 20.0, 1.0) for k in range(V)])
    grads = rng.standard_normal((K, V, 6)).astype(np.float32)
    P = torch.tensor(poses, device=DEV)
    m = torch.zeros((V, 6), device=DEV)
    v = torch.zeros((V, 6), device=DEV)
    st = torch.zeros(V, dtype=torch.int32, device=DEV)
    for it in range(K):
        before = P.cpu().numpy().astype(np.float64)
        mb, vb = m.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)
        R.pose_adam(P, torch.tensor(grads[it], device=DEV), m, v, st, 1e-2, 1e-2, K,
                    parametrization="t_so3")
        got = P.cpu().numpy()
        for k in range(V):
            ref, mm, vv, _ = PV.pose_adam_txso3(before[k], mb[k], vb[k], grads[it][k], it + 1, 1e-2,
                                                beta1=float(np.float32(0.9)),
                                                beta2=float(np.float32(0.999)),
                                                eps=float(np.float32(1e-8)))
            assert np.max(np.abs(got[k] - ref)) <= 2e-6, (it, k)
            assert np.max(np.abs(m.cpu().numpy()[k] - mm)) <= 1e-6 * max(1.0, np.max(np.abs(mm)))


def _tiny_target():
    wl = S.tiny()
    cam = wl.camera
    g = R.GaussianParams.from_set(wl.scene, DEV)
    rast = R.Rasterizer(0)
    target, _ = rast.forward(g, [cam], torch.tensor(wl.pose[None], device=DEV))
    return wl, cam, g, target.clone()


@pytest.mark.parametrize("param", ["se3", "t_so3"])
def test_solve_converges_in_both_parametrisations(param):
    wl, cam, g, target = _tiny_target()
    init = torch.tensor(wl.init_pose[None], device=DEV)
    pose = R.solve_poses(g, [cam], target, init, steps=150, lr=(1e-2, 1e-4), parametrization=param)
    e0 = S.pose_error(wl.init_pose, wl.pose)
    e1 = S.pose_error(pose[0].cpu().numpy(), wl.pose)
    assert e1[0] < 0.1 * e0[0] and e1[1] < 0.1 * e0[1], (param, e0, e1)


def test_multi_hypothesis_picks_the_converged_start():
    wl, cam, g, target = _tiny_target()
    rng = S.rng_for(77, 1)
    inits = [S.perturb_pose(wl.pose, 40.0, 0.8, rng) for _ in range(5)]
    inits.insert(3, wl.init_pose.astype(np.float64))     # the one near start (2 deg / 0.05)
    inits = torch.tensor(np.stack(inits).astype(np.float32), device=DEV)
    best, idx, losses, poses = R.solve_multi_hypothesis(g, cam, target, inits, steps=150)
    assert idx == 3, losses.cpu().numpy()
    e = S.pose_error(best.cpu().numpy(), wl.pose)
    assert e[0] < 0.2 and e[1] < 0.005, e
    # each hypothesis is the same solve it would be alone
    alone = R.solve_poses(g, [cam], target, inits[3:4].contiguous(), steps=150)
    assert torch.equal(alone[0], poses[3])
