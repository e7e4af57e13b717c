"""Relative pose estimation between two nearby frames (Sec. III-D), every
step on the device.

Frame t's depth map is unprojected into isotropic Gaussians
(gsp_unproject: pixel colour, three-nearest-neighbour scale), the scene is
fitted to frame t with L_RGB (JointRefiner, poses held), and the pose of
frame t+1 relative to frame t is solved with the confidence-masked L1 of
Eq. (20)-(21) (solve_poses(masked=True)).
"""
import ctypes
from typing import Optional

import torch

from . import _native as N
from .joint import JointHyper, JointRefiner, RawGaussians
from .render import _ptr, _stream, context, solve_poses


def unproject(cam, depth: torch.Tensor, image: torch.Tensor, stride: int = 4,
              opacity: float = 0.5, sh_degree: int = 0) -> RawGaussians:
    """Raw Gaussians of frame t from its depth map [h, w] and image [3, h, w]
    (device FP32, over the camera's region of interest)."""
    L = N.lib()
    view = N.view_array([cam])
    n = ctypes.c_int64()
    N.check(L.gsp_unproject_count(view, int(stride), ctypes.byref(n)), "gsp_unproject_count")
    n = n.value
    dev = depth.device
    S = (sh_degree + 1) ** 2
    raw = RawGaussians(torch.empty((n, 3), device=dev), torch.empty((n, 3), device=dev),
                       torch.empty((n, 4), device=dev), torch.empty(n, device=dev),
                       torch.empty((n, S, 3), device=dev), int(sh_degree))
    scratch = torch.empty(L.gsp_unproject_scratch_bytes(view, int(stride)), dtype=torch.uint8,
                          device=dev)
    prm = raw.struct()
    N.check(L.gsp_unproject(context(dev.index), view, _ptr(depth.contiguous()),
                            _ptr(image.contiguous()), int(stride), float(opacity), int(sh_degree),
                            ctypes.byref(prm), _ptr(scratch), scratch.numel(), _stream()),
            "gsp_unproject")
    return raw


def identity_poses(k, device):
    p = torch.zeros((k, 3, 4), device=device)
    p[:, 0, 0] = p[:, 1, 1] = p[:, 2, 2] = 1.0
    return p


FIT_HYPER = JointHyper(lr_means=(1.6e-4, 1.6e-6))


def relative_pose(cam, image_t: torch.Tensor, depth_t: torch.Tensor, image_t1: torch.Tensor,
                  stride: int = 4, fit_steps: int = 100, pose_steps: int = 200,
                  lr=(1e-3, 1e-4), hp: Optional[JointHyper] = None, init=None,
                  opacity: float = 0.5):
    """(pose of frame t+1 relative to frame t [3, 4], fitted raw scene of
    frame t).  Frame t's camera is the world frame.  The fit of frame t's
    scene (100 steps, Sec. IV) keeps the means nearly in place (FIT_HYPER:
    1.6e-4 -> 1.6e-6) so that the geometry stays the depth map's; the pose
    solve runs on the masked L1 for 200 steps at a learning rate decaying
    from 1e-3 to 1e-4 on a cosine schedule, the settings Sec. IV gives for
    the relative pose between consecutive frames."""
    dev = image_t.device
    hp = hp or FIT_HYPER
    raw = unproject(cam, depth_t, image_t, stride, opacity=opacity)
    ident = identity_poses(1, dev)
    ref = JointRefiner(raw, [cam], [image_t.view(3, cam.height, cam.width)], ident, fit_steps,
                       hp=hp, optimize_poses=False)
    for _ in range(fit_steps):
        ref.step()
    init = ident if init is None else init.reshape(1, 3, 4).contiguous()
    pose = solve_poses(ref.g, [cam], image_t1.reshape(-1).contiguous(), init, steps=pose_steps,
                       lr=lr, masked=True)
    return pose[0], raw
