"""Pins of the T x SO(3) pose oracle (oracle/pose_variants.py): Rodrigues
against scipy's matrix exponential, the gradient mapping against central
differences of a smooth function of the pose through both perturbations
(the SE(3) one by the C oracle's retraction), and the step against
torch.optim.Adam."""
import numpy as np
import scipy.linalg
import torch

import oracle
from oracle import pose_variants as PV


def _skew(p):
    return np.array([[0.0, -p[2], p[1]], [p[2], 0.0, -p[0]], [-p[1], p[0], 0.0]])


def _pose(seed):
    rng = np.random.default_rng(seed)
    R = scipy.linalg.expm(_skew(rng.normal(0, 0.7, 3)))
    return np.concatenate([R, rng.normal(0, 1, (3, 1))], axis=1)


def test_so3_exp_matches_expm():
    rng = np.random.default_rng(1)
    for s in (1e-9, 1e-3, 0.5, 2.5):
        phi = rng.normal(0, 1, 3)
        phi *= s / np.linalg.norm(phi)
        assert np.max(np.abs(PV.so3_exp(phi) - scipy.linalg.expm(_skew(phi)))) < 1e-14


def _objective(pose):
    # any smooth function of R and t
    R, t = pose[:, :3], pose[:, 3]
    w = np.array([[0.3, -1.2, 0.7], [2.0, 0.1, -0.4], [0.5, 0.9, 1.1]])
    return float(np.sum(w * R) + np.sin(t) @ np.array([1.0, -2.0, 0.5]) + (t @ t) * 0.3)


def test_gradient_mapping_by_differences():
    pose = _pose(2)
    h = 1e-6
    # left-twist gradient through the C oracle's SE(3) retraction
    g = np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        g[k] = (_objective(oracle.se3_retract(e, pose)) - _objective(oracle.se3_retract(-e, pose))) / (2 * h)
    # gradient in (c, phi) by perturbing the centre and rotating about it
    R, t = pose[:, :3], pose[:, 3]
    c = -R.T @ t
    ref = np.zeros(6)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        pp = np.concatenate([R, (-R @ (c + e))[:, None]], axis=1)
        pm = np.concatenate([R, (-R @ (c - e))[:, None]], axis=1)
        ref[k] = (_objective(pp) - _objective(pm)) / (2 * h)
        Rp, Rm = PV.so3_exp(e) @ R, PV.so3_exp(-e) @ R
        pp = np.concatenate([Rp, (-Rp @ c)[:, None]], axis=1)
        pm = np.concatenate([Rm, (-Rm @ c)[:, None]], axis=1)
        ref[3 + k] = (_objective(pp) - _objective(pm)) / (2 * h)
    assert np.max(np.abs(PV.txso3_gradient(pose, g) - ref)) < 1e-8


def test_step_matches_torch_adam_and_keeps_centre_under_rotation():
    pose = _pose(3)
    m = np.zeros(6)
    v = np.zeros(6)
    x = torch.zeros(6, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([x], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    rng = np.random.default_rng(4)
    for k in range(1, 5):
        g = rng.normal(0, 1, 6)
        new, m, v, delta = PV.pose_adam_txso3(pose, m, v, g, k, 1e-2)
        before = x.detach().clone()
        x.grad = torch.tensor(PV.txso3_gradient(pose, g))
        opt.step()
        assert np.max(np.abs((x.detach() - before).numpy() - delta)) < 1e-15
        c0 = -pose[:, :3].T @ pose[:, 3]
        c1 = -new[:, :3].T @ new[:, 3]
        assert np.max(np.abs(c1 - (c0 + delta[:3]))) < 1e-13
        assert np.max(np.abs(new[:, :3] - PV.so3_exp(delta[3:]) @ pose[:, :3])) < 1e-14
        pose = new
    # a rotation-only gradient leaves the centre where it is
    new, _, _, _ = PV.pose_adam_txso3(pose, np.zeros(6), np.zeros(6), np.array([0, 0, 0, 1.0, -2, 0.5]), 1, 1e-2)
    assert np.max(np.abs(-new[:, :3].T @ new[:, 3] - (-pose[:, :3].T @ pose[:, 3]))) < 1e-13
