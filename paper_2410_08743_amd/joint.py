"""Joint reconstruction and pose refinement (Sec. III-C) with every step on
the device.

One refinement step over a batch of views: render (gsp_render_fwd), the image
loss L_RGB = (1 - beta) L1 + beta DSSIM of Eq. (16) and its gradient
(gsp_loss_rgb), every Gaussian gradient and the views' pose twists
(gsp_render_bwd), Adam on the raw Gaussian parameters with the anisotropy
hinge L_An of Eq. (17) (gsp_gaussian_adam) and tangent-space Adam on the
batch's poses (gsp_pose_adam).  The losses of a batch's views are summed
(Eq. (14)).  Nothing synchronises with the host inside a step; an
instance-capacity overflow makes both Adam kernels skip that step on the
device, and `overflowed()` reports it afterwards.
"""
import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _native as N
from .render import GaussianParams, Rasterizer, _ptr, _stream, context, pose_adam, view_ptrs


@dataclass
class RawGaussians:
    """Raw (optimised) Gaussian parameters on the device, FP32 contiguous:
    scales = exp(log_scales), opacities = sigmoid(logit_opacities)."""
    means: torch.Tensor            # [n, 3]
    log_scales: torch.Tensor       # [n, 3]
    quats: torch.Tensor            # [n, 4]
    logit_opacities: torch.Tensor  # [n]
    sh: torch.Tensor               # [n, S, 3]
    sh_degree: int

    @property
    def n(self):
        return int(self.means.shape[0])

    @staticmethod
    def from_set(gs, device="cuda"):
        """From activated parameters (scales > 0, opacities in (0, 1))."""
        f = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float32)).to(device).contiguous()
        op = np.asarray(gs.opacities, dtype=np.float64)
        return RawGaussians(f(gs.means), f(np.log(np.asarray(gs.scales, dtype=np.float64))),
                            f(gs.quats), f(np.log(op) - np.log1p(-op)), f(gs.sh),
                            int(gs.sh_degree))

    def struct(self):
        for name in ("means", "log_scales", "quats", "logit_opacities", "sh"):
            t = getattr(self, name)
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous float32 device tensor")
        return N.GaussianParams(self.means.data_ptr(), self.log_scales.data_ptr(),
                                self.quats.data_ptr(), self.logit_opacities.data_ptr(),
                                self.sh.data_ptr())


@dataclass
class JointHyper:
    """Step sizes of the joint refinement: the means' rate decays
    exponentially (Sec. IV: 1.6e-2 -> 1.6e-4, not scaled by the scene
    extent), the camera rate follows a cosine decay 1e-2 -> 1e-4, the other
    groups keep the constant rates of 3DGS."""
    lr_means: tuple = (1.6e-2, 1.6e-4)
    lr_sh_dc: float = 2.5e-3
    lr_sh_rest: float = 2.5e-3 / 20
    lr_opacities: float = 5e-2
    lr_scales: float = 5e-3
    lr_quats: float = 1e-3
    betas: tuple = (0.9, 0.999)
    eps: float = 1e-15
    aniso_r: float = 10.0
    aniso_weight: float = 1.0
    beta_ssim: float = 0.2
    lr_pose: tuple = (1e-2, 1e-4)
    pose_eps: float = 1e-8

    def struct(self, total_steps):
        return N.GaussianAdamParams(self.lr_means[0], self.lr_means[1], int(total_steps),
                                    self.lr_sh_dc, self.lr_sh_rest, self.lr_opacities,
                                    self.lr_scales, self.lr_quats, self.betas[0], self.betas[1],
                                    self.eps, self.aniso_r, self.aniso_weight)


def loss_rgb(cams: Sequence, pred, target, grad=None, beta: float = 0.2, with_loss: bool = True,
             scratch: Optional[torch.Tensor] = None):
    """(per-view L_RGB [V] or None, grad).  pred, target, grad: packed tensors
    (views one after another) or lists of per-view tensors."""
    L = N.lib()
    views = N.view_array(cams)
    if grad is None:
        grad = ([torch.empty_like(p) for p in pred] if isinstance(pred, (list, tuple))
                else torch.empty_like(pred))
    dev = (pred[0] if isinstance(pred, (list, tuple)) else pred).device
    need = L.gsp_loss_rgb_scratch_bytes(len(cams), views)
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(need, dtype=torch.uint8, device=dev)
    loss = torch.empty(len(cams), dtype=torch.float32, device=dev) if with_loss else None
    N.check(L.gsp_loss_rgb(context(dev.index), len(cams), views, view_ptrs(pred, cams, 3),
                           view_ptrs(target, cams, 3), view_ptrs(grad, cams, 3), _ptr(loss),
                           float(beta), _ptr(scratch), scratch.numel(), _stream()), "gsp_loss_rgb")
    return loss, grad


def moments_size(n, sh_degree):
    return n * (11 + 3 * (sh_degree + 1) ** 2)


def gaussian_adam(raw: RawGaussians, grads: dict, m, v, step: int, total_steps: int,
                  hp: JointHyper, scales_out, opacities_out, aniso_loss=None, scratch=None,
                  guard=None):
    """One Adam step on `raw` in place; scales_out / opacities_out receive the
    activated values; aniso_loss (device float [1]) receives L_An before the
    step."""
    L = N.lib()
    gr = N.Grads(*[grads[k].data_ptr() for k in ("means", "scales", "quats", "opacities", "sh")],
                 None)
    if aniso_loss is not None:
        need = L.gsp_gaussian_adam_scratch_bytes(raw.n)
        if scratch is None or scratch.numel() < need:
            scratch = torch.empty(need, dtype=torch.uint8, device=raw.means.device)
    prm = raw.struct()
    hps = hp.struct(total_steps)
    N.check(L.gsp_gaussian_adam(context(raw.means.device.index), raw.n, raw.sh_degree,
                                ctypes.byref(prm), ctypes.byref(gr), _ptr(m), _ptr(v), int(step),
                                ctypes.byref(hps), _ptr(scales_out), _ptr(opacities_out),
                                _ptr(aniso_loss), _ptr(scratch), _ptr(guard), _stream()),
            "gsp_gaussian_adam")


class JointRefiner:
    """Joint refinement of a Gaussian scene and the poses of K views.

    cams, targets: K cameras and [3, h, w] target images; init_poses [K, 3, 4]
    (world->camera).  Views are visited in batches of `views_per_step`
    consecutive views of `order` (default 0..K-1), cycling; each batch's
    poses, moments and step counts are contiguous, so no gathers run in a
    step.  The instance capacity is sized once from renders of every batch at
    the initial state with `margin`.
    """

    def __init__(self, raw: RawGaussians, cams: Sequence, targets: Sequence[torch.Tensor],
                 init_poses: torch.Tensor, total_steps: int, views_per_step: int = 1,
                 hp: Optional[JointHyper] = None, order: Optional[Sequence[int]] = None,
                 margin: float = 1.5, rast: Optional[Rasterizer] = None,
                 optimize_poses: bool = True):
        self.raw = raw
        self.optimize_poses = bool(optimize_poses)
        self.hp = hp or JointHyper()
        K = len(cams)
        order = list(range(K)) if order is None else [int(i) for i in order]
        self.order = order
        self.cams = [cams[i] for i in order]
        self.targets = [targets[i].contiguous() for i in order]
        dev = raw.means.device
        self.dev = dev
        self.poses = init_poses[order].contiguous().clone()
        self.V = int(views_per_step)
        self.batches = [(i, min(i + self.V, K)) for i in range(0, K, self.V)]
        self.total_steps = int(total_steps)
        visits = -(-self.total_steps * self.V // K)
        self.pose_steps_total = max(1, visits)
        n, deg = raw.n, raw.sh_degree
        S = (deg + 1) ** 2
        self.m = torch.zeros(moments_size(n, deg), device=dev)
        self.v = torch.zeros(moments_size(n, deg), device=dev)
        self.scales = torch.exp(raw.log_scales).contiguous()
        self.opacities = torch.sigmoid(raw.logit_opacities).contiguous()
        self.g = GaussianParams(raw.means, self.scales, raw.quats, self.opacities, raw.sh, deg)
        self.pm = torch.zeros((K, 6), device=dev)
        self.pv = torch.zeros((K, 6), device=dev)
        self.psteps = torch.zeros(K, dtype=torch.int32, device=dev)
        self.grads = {"means": torch.empty((n, 3), device=dev), "scales": torch.empty((n, 3), device=dev),
                      "quats": torch.empty((n, 4), device=dev), "opacities": torch.empty(n, device=dev),
                      "sh": torch.empty((n, S, 3), device=dev),
                      "pose": torch.empty((self.V, 6), device=dev)}
        # one buffer per position in a batch, large enough for every view
        # that takes that position (views may differ in size)
        npix = lambda c: 3 * (c.roi[2] * c.roi[3] if getattr(c, "roi", None) else c.width * c.height)
        sizes = [max(npix(self.cams[a + j]) for a, b in self.batches if a + j < b)
                 for j in range(self.V)]
        self.images = [torch.empty(n, device=dev) for n in sizes]
        self.dl = [torch.empty(n, device=dev) for n in sizes]
        self.aniso = torch.zeros(1, device=dev)
        self.loss = torch.zeros(self.V, device=dev)
        L = N.lib()
        self.loss_scratch = torch.empty(max(L.gsp_loss_rgb_scratch_bytes(b - a, N.view_array(self.cams[a:b]))
                                            for a, b in self.batches), dtype=torch.uint8, device=dev)
        self.adam_scratch = torch.empty(L.gsp_gaussian_adam_scratch_bytes(n), dtype=torch.uint8,
                                        device=dev)
        self.rast = rast or Rasterizer(dev.index)
        cap = 0
        for a, b in self.batches:
            self.rast.forward(self.g, self.cams[a:b], self.poses[a:b])
            cap = max(cap, self.rast.instances()[0])
        self.rast.capacity = int(margin * cap) + 4096
        self.rast.ws = None
        for a, b in self.batches:     # room for the largest batch
            self.rast._ensure(self.g, N.view_array(self.cams[a:b]))
        self.k = 0

    def step(self, with_loss: bool = False):
        """One refinement step on the next batch of views."""
        a, b = self.batches[self.k % len(self.batches)]
        self.k += 1
        cams = self.cams[a:b]
        V = b - a
        poses = self.poses[a:b]
        npix = lambda c: 3 * (c.roi[2] * c.roi[3] if getattr(c, "roi", None) else c.width * c.height)
        imgs = [self.images[j][:npix(c)] for j, c in enumerate(cams)]
        dls = [self.dl[j][:npix(c)] for j, c in enumerate(cams)]
        self.rast.forward(self.g, cams, poses, check=False, images=imgs)
        view_losses, _ = loss_rgb(cams, imgs, self.targets[a:b], grad=dls, beta=self.hp.beta_ssim,
                                  with_loss=with_loss, scratch=self.loss_scratch)
        out = dict(self.grads)
        if self.optimize_poses:
            out["pose"] = self.grads["pose"][:V]
        else:
            del out["pose"]
        self.rast.backward(self.g, cams, poses, dls, pose=self.optimize_poses, out=out)
        gaussian_adam(self.raw, self.grads, self.m, self.v, self.k, self.total_steps, self.hp,
                      self.scales, self.opacities, aniso_loss=self.aniso if with_loss else None,
                      scratch=self.adam_scratch, guard=self.rast.ws)
        if self.optimize_poses:
            pose_adam(poses, out["pose"], self.pm[a:b], self.pv[a:b], self.psteps[a:b],
                      self.hp.lr_pose[0], self.hp.lr_pose[1], self.pose_steps_total,
                      self.hp.betas[0], self.hp.betas[1], self.hp.pose_eps, guard=self.rast.ws)
        if with_loss:
            return view_losses.sum() + self.aniso[0]
        return None

    def overflowed(self):
        return self.rast.overflowed()

    def poses_in_input_order(self):
        out = torch.empty_like(self.poses)
        out[self.order] = self.poses
        return out
