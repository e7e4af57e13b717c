"""PyTorch-facing layer over libgsp: device tensors in, device tensors out.

PyTorch provides device memory and the current HIP stream; every step of the
render, the loss, the backward and the pose update runs in the library's
kernels (include/gsp.h).

Main entry points:
  Rasterizer            workspace owner; forward / backward / loss / Adam calls
  render(...)           torch.autograd.Function: image from Gaussians and
                        pose twists tau (gradient = left se(3) twist, Sec. III-B)
  solve_poses(...)      tangent-space Adam pose estimation, all on device
"""
import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _native as N


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_contexts = {}


def context(device: int):
    """Library context of a device (created once per process)."""
    if device not in _contexts:
        L = N.lib()
        h = ctypes.c_void_p()
        N.check(L.gsp_create(int(device), ctypes.byref(h)), "gsp_create")
        _contexts[device] = h
    return _contexts[device]


@dataclass
class GaussianParams:
    """Activated Gaussian parameters on the device (FP32, contiguous)."""
    means: torch.Tensor      # [n, 3]
    scales: torch.Tensor     # [n, 3]
    quats: torch.Tensor      # [n, 4]
    opacities: torch.Tensor  # [n]
    sh: torch.Tensor         # [n, S, 3]
    sh_degree: int

    @property
    def n(self):
        return int(self.means.shape[0])

    @staticmethod
    def from_set(gs, device="cuda"):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).to(device).contiguous()
        return GaussianParams(f(gs.means), f(gs.scales), f(gs.quats), f(gs.opacities),
                              f(gs.sh), int(gs.sh_degree))

    def struct(self):
        for name in ("means", "scales", "quats", "opacities", "sh"):
            t = getattr(self, name)
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous float32 device tensor")
        return N.Gaussians(self.means.data_ptr(), self.scales.data_ptr(), self.quats.data_ptr(),
                           self.opacities.data_ptr(), self.sh.data_ptr(), self.n, self.sh_degree)


def region(cam):
    return cam.roi if getattr(cam, "roi", None) is not None else (0, 0, cam.width, cam.height)


def pixel_counts(cams):
    return [region(c)[2] * region(c)[3] for c in cams]


def split_images(packed, cams):
    """Per-view [3, h, w] views of a packed image buffer."""
    out, off = [], 0
    for c in cams:
        _, _, w, h = region(c)
        out.append(packed[off:off + 3 * w * h].view(3, h, w))
        off += 3 * w * h
    return out


def pack_images(images):
    return torch.cat([im.reshape(-1) for im in images]).contiguous()


def view_ptrs(buf, cams, channels):
    """Device pointers of each view's `channels` x h x w block: `buf` is either
    one packed tensor (views one after another) or a list of per-view
    tensors."""
    if buf is None:
        return None
    if isinstance(buf, (list, tuple)):
        if len(buf) != len(cams):
            raise ValueError("one tensor per view expected")
        out = []
        for t, c in zip(buf, cams):
            _, _, w, h = region(c)
            if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != channels * w * h:
                raise ValueError(f"per-view tensor must be contiguous float32 with {channels}*h*w values")
            out.append(t.data_ptr())
        return N.ptr_array(out)
    if buf.dtype != torch.float32 or not buf.is_contiguous():
        raise ValueError("packed buffer must be contiguous float32")
    counts = [channels * n for n in pixel_counts(cams)]
    if buf.numel() < sum(counts):
        raise ValueError("packed buffer too small for the views")
    out, off = [], 0
    for n in counts:
        out.append(buf.data_ptr() + 4 * off)
        off += n
    return N.ptr_array(out)


class Rasterizer:
    """Owns the device workspace of a sequence of renders.

    The workspace is sized for an instance capacity (number of (Gaussian,
    tile) pairs).  With check=True a forward synchronises once to read the
    instance count and re-runs with a larger capacity on overflow; with
    check=False nothing synchronises and `overflowed()` tells afterwards
    whether any forward since the workspace was allocated ran out of room.

    With store_lists=True (GSP_STORE_LISTS) every forward also stores each
    pixel's blended entries (list position, alpha, transmittance in front;
    12 bytes per blended pair, in a second buffer sized for `pair_capacity`
    pairs and grown like the workspace), and the backward reads them instead
    of recomputing the compositing.
    """

    def __init__(self, device: Optional[int] = None, capacity: int = 0, growth: float = 1.5,
                 store_lists: bool = False, pair_capacity: int = 0):
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.capacity = int(capacity)
        self.growth = float(growth)
        self.store_lists = bool(store_lists)
        self.pair_capacity = int(pair_capacity)
        self.lists = None
        self.ws = None
        # incremented by every forward: an autograd context remembers the
        # generation of its forward and refuses to back-propagate once the
        # workspace holds another forward's state
        self.generation = 0

    # -- workspace ---------------------------------------------------------
    def _ws_bytes(self, n, degree, views, cap):
        L = N.lib()
        sz = ctypes.c_size_t()
        N.check(L.gsp_workspace_size(n, degree, len(views), views, cap, ctypes.byref(sz)),
                "gsp_workspace_size")
        return sz.value

    def _ensure(self, g, views):
        nbytes = self._ws_bytes(g.n, g.sh_degree, views, self.capacity)
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = torch.zeros(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
        return nbytes

    def _lists_bytes(self, views):
        return N.lib().gsp_lists_bytes(len(views), views, self.pair_capacity)

    def _ensure_lists(self, views):
        nbytes = self._lists_bytes(views)
        if nbytes == 0:
            raise ValueError("bad views or pair capacity for the stored lists")
        if self.lists is None or self.lists.numel() < nbytes:
            self.lists = torch.zeros(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
        return nbytes

    def reset_overflow(self):
        if self.ws is not None:
            self.ws[:64].zero_()
        if self.lists is not None:
            self.lists[:64].zero_()

    def instances(self):
        """(M of the last forward, overflow flag); synchronises the stream."""
        L = N.lib()
        m = ctypes.c_int64()
        o = ctypes.c_int32()
        N.check(L.gsp_instances(context(self.device), _ptr(self.ws), _stream(), ctypes.byref(m),
                                ctypes.byref(o)), "gsp_instances")
        return m.value, bool(o.value)

    def list_pairs(self):
        """(stored pairs of the last forward, overflow flag of the pair
        capacity); store_lists mode only; synchronises the stream."""
        L = N.lib()
        q = ctypes.c_int64()
        o = ctypes.c_int32()
        N.check(L.gsp_list_pairs(context(self.device), _ptr(self.lists), _stream(),
                                 ctypes.byref(q), ctypes.byref(o)), "gsp_list_pairs")
        return q.value, bool(o.value)

    def overflowed(self):
        ovf = self.instances()[1]
        if self.store_lists and self.lists is not None:
            ovf = ovf or self.list_pairs()[1]
        return ovf

    # -- forward / backward ------------------------------------------------
    def forward(self, g: GaussianParams, cams: Sequence, poses: torch.Tensor,
                alphas=False, check: bool = True, images=None):
        """Renders len(cams) views; returns (images, alphas or None).
        `alphas`: False, True (a packed tensor of 1 - T_final is made) or an
        output buffer (packed tensor or list of per-view [h, w] tensors).
        `images` is an optional output: one packed tensor or a list of
        per-view [3, h, w] tensors; by default a packed tensor is made."""
        images, al, _ = self._forward(g, cams, poses, alphas, check, images, None, False)
        return images, al

    def forward_l1(self, g: GaussianParams, cams: Sequence, poses: torch.Tensor, targets,
                   grad=None, with_loss: bool = False, alphas=False, check: bool = True):
        """Render and L1 loss in one pass (gsp_render_fwd_l1): returns
        (per-view losses [V] or None, dL/dimage, alphas or None).  The
        gradient is the one loss_l1 computes from the rendered images, bit for
        bit; the images themselves are not kept.  `targets` and `grad` are
        packed tensors or lists of per-view [3, h, w] tensors."""
        grad, al, loss = self._forward(g, cams, poses, alphas, check, grad, targets, with_loss)
        return loss, grad, al

    def _forward(self, g, cams, poses, alphas, check, images, targets, with_loss):
        L = N.lib()
        views = N.view_array(cams)
        poses = poses.contiguous()
        if poses.dtype != torch.float32 or tuple(poses.shape) != (len(cams), 3, 4):
            raise ValueError("poses must be float32 [V, 3, 4]")
        P = sum(pixel_counts(cams))
        dev = f"cuda:{self.device}"
        if images is None:
            images = torch.empty(3 * P, dtype=torch.float32, device=dev)
        if isinstance(alphas, bool):
            al = torch.empty(P, dtype=torch.float32, device=dev) if alphas else None
        else:
            al = alphas
        if self.capacity <= 0:
            self.capacity = max(1024, 8 * g.n * len(cams))
        if self.store_lists and self.pair_capacity <= 0:
            self.pair_capacity = 32 * P + 1024
        gs = g.struct()
        img_ptrs = view_ptrs(images, cams, 3)
        al_ptrs = view_ptrs(al, cams, 1)
        loss = None
        if targets is not None:
            if self.store_lists:
                raise ValueError("the L1-fused forward does not store lists")
            tgt_ptrs = view_ptrs(targets, cams, 3)
            if with_loss:
                loss = torch.empty(len(cams), dtype=torch.float32, device=dev)
        for _ in range(8):
            nbytes = self._ensure(g, views)
            if targets is not None:
                N.check(L.gsp_render_fwd_l1(context(self.device), ctypes.byref(gs), len(cams),
                                            views, _ptr(poses), tgt_ptrs, img_ptrs, al_ptrs,
                                            _ptr(loss), _ptr(self.ws), nbytes, self.capacity,
                                            _stream()), "gsp_render_fwd_l1")
            elif self.store_lists:
                lbytes = self._ensure_lists(views)
                N.check(L.gsp_render_fwd_store(context(self.device), ctypes.byref(gs), len(cams),
                                               views, _ptr(poses), img_ptrs, al_ptrs, _ptr(self.ws),
                                               nbytes, self.capacity, _ptr(self.lists), lbytes,
                                               self.pair_capacity, _stream()),
                        "gsp_render_fwd_store")
            else:
                N.check(L.gsp_render_fwd(context(self.device), ctypes.byref(gs), len(cams), views,
                                         _ptr(poses), img_ptrs, al_ptrs, _ptr(self.ws), nbytes,
                                         self.capacity, _stream()), "gsp_render_fwd")
            if not check:
                break
            m, ovf = self.instances()
            if ovf:
                self.capacity = int(m * self.growth) + 1024
                self.ws = None       # reallocated (zeroed) at the larger size
                continue
            if self.store_lists:
                q, lovf = self.list_pairs()
                if lovf:
                    self.pair_capacity = int(q * self.growth) + 1024
                    self.lists = None
                    continue
            break
        self.generation += 1
        return images, al, loss

    def backward(self, g: GaussianParams, cams: Sequence, poses: torch.Tensor,
                 dl_dimages, want=("means", "scales", "quats", "opacities", "sh"),
                 pose: bool = True, accumulate: bool = False, out=None):
        """Gradients of the last forward.  `dl_dimages` is packed like the
        images or a list of per-view tensors.  Returns a dict with the
        requested Gaussian gradients and 'pose' ([V, 6], left twist (rho, phi))."""
        L = N.lib()
        views = N.view_array(cams)
        dev = f"cuda:{self.device}"
        out = dict(out or {})
        shapes = {"means": (g.n, 3), "scales": (g.n, 3), "quats": (g.n, 4),
                  "opacities": (g.n,), "sh": tuple(g.sh.shape)}
        for k in want:
            if k not in out:
                out[k] = torch.empty(shapes[k], dtype=torch.float32, device=dev)
        if pose and "pose" not in out:
            out["pose"] = torch.empty((len(cams), 6), dtype=torch.float32, device=dev)
        gr = N.Grads(*[out[k].data_ptr() if k in out else None
                       for k in ("means", "scales", "quats", "opacities", "sh", "pose")])
        gs = g.struct()
        nbytes = self._ws_bytes(g.n, g.sh_degree, views, self.capacity)
        flags = N.GSP_ACCUMULATE if accumulate else 0
        if self.store_lists:
            N.check(L.gsp_render_bwd_stored(context(self.device), ctypes.byref(gs), len(cams),
                                            views, _ptr(poses.contiguous()),
                                            view_ptrs(dl_dimages, cams, 3), _ptr(self.ws), nbytes,
                                            self.capacity, _ptr(self.lists),
                                            self._lists_bytes(views), self.pair_capacity,
                                            ctypes.byref(gr), flags, _stream()),
                    "gsp_render_bwd_stored")
        else:
            N.check(L.gsp_render_bwd(context(self.device), ctypes.byref(gs), len(cams), views,
                                     _ptr(poses.contiguous()), view_ptrs(dl_dimages, cams, 3),
                                     _ptr(self.ws), nbytes, self.capacity, ctypes.byref(gr), flags,
                                     _stream()), "gsp_render_bwd")
        return out

    def backward_pose_step(self, g: GaussianParams, cams: Sequence, poses: torch.Tensor, dl_dimages,
                           dpose, m, v, steps, lr_start, lr_end, total_steps, beta1=0.9,
                           beta2=0.999, eps=1e-8, parametrization: str = "se3"):
        """The pose-only backward of the last forward followed by the Adam
        step of `pose_adam` (guarded by this workspace), in the backward's
        launches: `dpose` receives the pose gradient and `poses`, `m`, `v`,
        `steps` are updated in place, bit for bit as the two calls would."""
        if self.store_lists:
            raise ValueError("backward_pose_step runs the recomputing backward only")
        L = N.lib()
        views = N.view_array(cams)
        gs = g.struct()
        nbytes = self._ws_bytes(g.n, g.sh_degree, views, self.capacity)
        prm = N.AdamParams(lr_start, lr_end, int(total_steps), beta1, beta2, eps,
                           PARAMETRIZATIONS[parametrization])
        if not poses.is_contiguous():
            raise ValueError("poses must be contiguous: they are updated in place")
        N.check(L.gsp_render_bwd_pose_step(context(self.device), ctypes.byref(gs), len(cams), views,
                                           _ptr(poses), view_ptrs(dl_dimages, cams, 3),
                                           _ptr(self.ws), nbytes, self.capacity, _ptr(dpose),
                                           _ptr(m), _ptr(v), _ptr(steps), ctypes.byref(prm),
                                           _stream()), "gsp_render_bwd_pose_step")

    def inspect(self, g: GaussianParams, cams: Sequence, name: str, dtype=torch.float32):
        """A copy of an intermediate workspace array of the last call."""
        L = N.lib()
        views = N.view_array(cams)
        gs = g.struct()
        nbytes = self._ws_bytes(g.n, g.sh_degree, views, self.capacity)
        p = ctypes.c_void_p()
        cnt = ctypes.c_int64()
        N.check(L.gsp_inspect(context(self.device), ctypes.byref(gs), len(cams), views,
                              _ptr(self.ws), nbytes, self.capacity, name.encode(), ctypes.byref(p),
                              ctypes.byref(cnt)), "gsp_inspect")
        itemsize = torch.empty((), dtype=dtype).element_size()
        base = self.ws.data_ptr()
        off = p.value - base
        elem_bytes = {"geom": 16, "color": 16, "rect": 8, "ranges": 8}.get(name, 4)
        nbytes_arr = cnt.value * elem_bytes
        raw = self.ws[off:off + nbytes_arr]
        return raw.view(dtype).clone() if nbytes_arr % itemsize == 0 else raw.clone()


def loss_l1(cams: Sequence, pred, target, grad=None, with_loss: bool = True):
    """(per-view losses [V] or None, grad): mean |pred - target| of each view
    and its gradient.  pred, target and grad are packed tensors (views one
    after another) or lists of per-view tensors."""
    L = N.lib()
    views = N.view_array(cams)
    if grad is None:
        grad = ([torch.empty_like(p) for p in pred] if isinstance(pred, (list, tuple))
                else torch.empty_like(pred))
    dev = (pred[0] if isinstance(pred, (list, tuple)) else pred).device
    loss = scratch = None
    if with_loss:
        loss = torch.empty(len(cams), dtype=torch.float32, device=dev)
        scratch = torch.empty(L.gsp_loss_l1_scratch_bytes(len(cams), views), dtype=torch.uint8,
                              device=dev)
    N.check(L.gsp_loss_l1(context(dev.index), len(cams), views, view_ptrs(pred, cams, 3),
                          view_ptrs(target, cams, 3), view_ptrs(grad, cams, 3), _ptr(loss),
                          _ptr(scratch), _stream()), "gsp_loss_l1")
    return loss, grad


def masked_l1(cams: Sequence, pred, target, alpha, grad=None, with_loss: bool = True,
              scratch: Optional[torch.Tensor] = None):
    """(per-view masked L1 sums [V] or None, grad) of Eq. (21) with the mask
    of Eq. (20) from the render's accumulated opacity `alpha` (packed or a
    list of per-view [h, w] tensors, as gsp_render_fwd writes it)."""
    L = N.lib()
    views = N.view_array(cams)
    if grad is None:
        grad = ([torch.empty_like(p) for p in pred] if isinstance(pred, (list, tuple))
                else torch.empty_like(pred))
    dev = (pred[0] if isinstance(pred, (list, tuple)) else pred).device
    loss = None
    if with_loss:
        loss = torch.empty(len(cams), dtype=torch.float32, device=dev)
        need = L.gsp_loss_masked_l1_scratch_bytes(len(cams), views)
        if scratch is None or scratch.numel() < need:
            scratch = torch.empty(need, dtype=torch.uint8, device=dev)
    N.check(L.gsp_loss_masked_l1(context(dev.index), len(cams), views, view_ptrs(pred, cams, 3),
                                 view_ptrs(target, cams, 3), view_ptrs(alpha, cams, 1),
                                 view_ptrs(grad, cams, 3), _ptr(loss),
                                 _ptr(scratch if with_loss else None), _stream()),
            "gsp_loss_masked_l1")
    return loss, grad


PARAMETRIZATIONS = {"se3": N.GSP_POSE_SE3, "t_so3": N.GSP_POSE_T_SO3}


def pose_adam(poses, dpose, m, v, steps, lr_start, lr_end, total_steps, beta1=0.9, beta2=0.999,
              eps=1e-8, guard: Optional[torch.Tensor] = None, parametrization: str = "se3"):
    """In-place tangent Adam step on every pose: in SE(3) with left
    retraction (the paper's), or with parametrization="t_so3" on the camera
    centre and the rotation separately; with a `guard` workspace whose last
    render overflowed, the step is skipped."""
    L = N.lib()
    prm = N.AdamParams(lr_start, lr_end, int(total_steps), beta1, beta2, eps,
                       PARAMETRIZATIONS[parametrization])
    N.check(L.gsp_pose_adam(context(poses.device.index), poses.shape[0], _ptr(poses), _ptr(dpose),
                            _ptr(m), _ptr(v), _ptr(steps), ctypes.byref(prm), _ptr(guard),
                            _stream()), "gsp_pose_adam")


def twist_apply(tau: torch.Tensor, poses: torch.Tensor, out: Optional[torch.Tensor] = None):
    """Exp(tau) poses per view (left perturbation; tau [V, 6] = (rho, phi),
    poses [V, 3, 4] world->camera)."""
    tau = tau.contiguous()
    poses = poses.contiguous()
    out = torch.empty_like(poses) if out is None else out
    N.check(N.lib().gsp_twist_apply(context(poses.device.index), poses.shape[0], _ptr(tau),
                                    _ptr(poses), _ptr(out), _stream()), "gsp_twist_apply")
    return out


def twist_chain(tau: torch.Tensor, dpose: torch.Tensor):
    """dL/dtau from the twist gradient at Exp(tau) poses: J(tau)^T dpose,
    J the left Jacobian of SE(3)."""
    tau = tau.contiguous()
    dpose = dpose.contiguous()
    out = torch.empty_like(dpose)
    N.check(N.lib().gsp_twist_chain(context(dpose.device.index), dpose.shape[0], _ptr(tau),
                                    _ptr(dpose), _ptr(out), _stream()), "gsp_twist_chain")
    return out


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacities, sh, tau, poses, cams, sh_degree, rast, check,
                apply_tau):
        g = GaussianParams(means.contiguous(), scales.contiguous(), quats.contiguous(),
                           opacities.contiguous(), sh.contiguous(), sh_degree)
        at = poses.detach().contiguous()
        if apply_tau:
            at = twist_apply(tau.detach(), at)
        images, _ = rast.forward(g, cams, at, check=check)
        ctx.g, ctx.cams, ctx.rast, ctx.generation = g, cams, rast, rast.generation
        ctx.apply_tau = apply_tau
        ctx.save_for_backward(at, tau.detach() if apply_tau else None)
        return images

    @staticmethod
    def backward(ctx, dl):
        at, tau = ctx.saved_tensors
        if ctx.rast.generation != ctx.generation:
            raise RuntimeError(
                "the Rasterizer rendered again after this forward, so its workspace no longer "
                "holds this forward's state; give each render whose backward is still pending "
                "its own Rasterizer")
        names = ("means", "scales", "quats", "opacities", "sh")
        want = tuple(k for k, need in zip(names, ctx.needs_input_grad[:5]) if need)
        need_pose = ctx.needs_input_grad[5]
        out = ctx.rast.backward(ctx.g, ctx.cams, at, dl.contiguous(), want=want, pose=need_pose)
        grads = [out.get(k) for k in names]
        dtau = out.get("pose")
        if dtau is not None and ctx.apply_tau:
            dtau = twist_chain(tau, dtau)
        return (*grads, dtau, None, None, None, None, None, None)


def render(g: GaussianParams, cams: Sequence, poses: torch.Tensor, tau: Optional[torch.Tensor] = None,
           rast: Optional[Rasterizer] = None, params=None, check: bool = True):
    """Differentiable render of len(cams) views; returns the packed images.

    `params` (optional) is a tuple (means, scales, quats, opacities, sh) of
    tensors that require grad; by default the tensors of `g` are used.  `tau`
    ([V, 6], (rho, phi) per view, optional) moves the poses: the views are
    rendered at Exp(tau) poses (the left perturbation of Sec. III-B), and
    tau.grad receives dL/dtau at the given tau (at tau = 0, the left se(3)
    twist gradient at `poses`; elsewhere chained through the left Jacobian of
    SE(3)), so tau may be optimised directly.  `poses` itself receives no
    gradient.  With check=False nothing synchronises; `rast.overflowed()`
    then tells afterwards whether any render ran out of instance capacity.
    """
    rast = rast or Rasterizer()
    apply_tau = tau is not None
    if tau is None:
        tau = torch.zeros((len(cams), 6), dtype=torch.float32, device=poses.device)
    p = params or (g.means, g.scales, g.quats, g.opacities, g.sh)
    return _RenderFn.apply(*p, tau, poses, list(cams), g.sh_degree, rast, check, apply_tau)


def solve_poses(g: GaussianParams, cams: Sequence, targets: torch.Tensor, init_poses: torch.Tensor,
                steps: int = 100, lr=(1e-2, 1e-4), betas=(0.9, 0.999), eps=1e-8,
                rast: Optional[Rasterizer] = None, history: bool = False, masked: bool = False,
                parametrization: str = "se3", final_loss: bool = False, graph: bool = False):
    """Estimates the poses of len(cams) views against packed target images by
    `steps` tangent-space Adam iterations on the L1 loss (cosine learning-rate
    decay lr[0] -> lr[1]); with masked=True on the confidence-masked L1 of
    Eq. (20)-(21) (pixels whose rendered opacity exceeds 0.99).
    `parametrization` is "se3" (the paper's) or "t_so3" (see pose_adam);
    with final_loss=True the per-view loss at the final poses is returned
    too (one more render).  Forward, loss, backward (pose only) and the update
    all run on the device without host synchronisation; the instance capacity
    is sized from the first render and the whole solve is repeated if any
    iteration overflowed it.  With graph=True one iteration is captured in a
    HIP graph and replayed `steps` times (no per-launch host work; the Adam
    step count and learning rate live on the device, so every replay is the
    next iteration); history is not available then."""
    if graph and history:
        raise ValueError("history is not recorded by a graph-replayed solve")
    rast = rast or Rasterizer()
    V = len(cams)
    dev = init_poses.device
    for _ in range(4):
        poses = init_poses.clone().contiguous()
        m = torch.zeros((V, 6), dtype=torch.float32, device=dev)
        v = torch.zeros((V, 6), dtype=torch.float32, device=dev)
        st = torch.zeros(V, dtype=torch.int32, device=dev)
        dpose = torch.zeros((V, 6), dtype=torch.float32, device=dev)
        P = sum(pixel_counts(cams))
        images = torch.empty(3 * P, dtype=torch.float32, device=dev)
        dl = torch.empty_like(images)
        alpha = torch.empty(P, dtype=torch.float32, device=dev) if masked else None
        mscratch = (torch.empty(N.lib().gsp_loss_masked_l1_scratch_bytes(V, N.view_array(cams)),
                                dtype=torch.uint8, device=dev) if masked and history else None)
        rast.forward(g, cams, poses, check=True, images=images)
        if rast.capacity < 1.5 * rast.instances()[0]:
            rast.capacity = int(1.5 * rast.instances()[0]) + 1024
            rast.ws = None
        rast._ensure(g, N.view_array(cams))
        rast.reset_overflow()
        hist = []

        def iteration():
            if masked:
                rast.forward(g, cams, poses, check=False, images=images, alphas=alpha)
                loss, _ = masked_l1(cams, images, targets, alpha, grad=dl, with_loss=history,
                                    scratch=mscratch)
            else:
                # render and L1 gradient in one pass
                loss, _, _ = rast.forward_l1(g, cams, poses, targets, grad=dl, with_loss=history,
                                             check=False)
            if rast.store_lists:
                rast.backward(g, cams, poses, dl, want=(), pose=True, out={"pose": dpose})
                pose_adam(poses, dpose, m, v, st, lr[0], lr[1], steps, betas[0], betas[1], eps,
                          guard=rast.ws, parametrization=parametrization)
            else:
                # the same step applied by the backward's final pose reduction
                rast.backward_pose_step(g, cams, poses, dl, dpose, m, v, st, lr[0], lr[1], steps,
                                        betas[0], betas[1], eps, parametrization=parametrization)
            return loss

        if graph:
            side = torch.cuda.Stream(device=dev)
            side.wait_stream(torch.cuda.current_stream(dev))
            cg = torch.cuda.CUDAGraph()
            with torch.cuda.graph(cg, stream=side):
                iteration()                 # recorded, not run
            for k in range(steps):
                cg.replay()
        else:
            for k in range(steps):
                loss = iteration()
                if history:
                    hist.append(loss)
        fin = None
        if final_loss:
            if masked:
                rast.forward(g, cams, poses, check=False, images=images, alphas=alpha)
                fin, _ = masked_l1(cams, images, targets, alpha, grad=dl)
            else:
                rast.forward(g, cams, poses, check=False, images=images)
                fin, _ = loss_l1(cams, images, targets, grad=dl)
        if not rast.overflowed():
            out = (poses,)
            if history:
                out += (torch.cat(hist).cpu().numpy(),)
            if final_loss:
                out += (fin,)
            return out if len(out) > 1 else poses
        rast.capacity = int(rast.capacity * rast.growth) + 1024
        rast.ws = None
    raise RuntimeError("instance capacity kept overflowing during the pose solve")


def solve_multi_hypothesis(g: GaussianParams, cam, target: torch.Tensor, inits: torch.Tensor,
                           steps: int = 100, lr=(1e-2, 1e-4), parametrization: str = "se3",
                           masked: bool = False, rast: Optional[Rasterizer] = None):
    """Pose estimation of one image from H starting poses at once: the H
    hypotheses are views of one launch (same camera, the one target image
    shared by pointer, no copies); returns (best pose [3, 4], index of the
    best hypothesis, final losses [H], all final poses [H, 3, 4]), best =
    lowest final loss."""
    H = int(inits.shape[0])
    targets = [target.reshape(-1)] * H
    poses, losses = solve_poses(g, [cam] * H, targets, inits.contiguous(), steps=steps, lr=lr,
                                rast=rast, masked=masked, parametrization=parametrization,
                                final_loss=True)
    best = int(torch.argmin(losses).item())
    return poses[best], best, losses, poses


PROFILE_TIMING = 1
PROFILE_COUNTS = 2


def profile_enable(device: int, mode: int):
    """Sets the library's measurement mode (bit mask of PROFILE_TIMING and
    PROFILE_COUNTS; 0 turns measurement off)."""
    N.check(N.lib().gsp_profile_enable(context(device), int(mode)), "gsp_profile_enable")


def profile_read(device: int, max_stages: int = 32):
    """{stage: (launches, total ms)} since the previous read; synchronises."""
    L = N.lib()
    names = ctypes.create_string_buffer(32 * max_stages)
    counts = (ctypes.c_int64 * max_stages)()
    ms = (ctypes.c_double * max_stages)()
    n = ctypes.c_int32()
    N.check(L.gsp_profile_read(context(device), max_stages, names, counts, ms, ctypes.byref(n)),
            "gsp_profile_read")
    out = {}
    for k in range(n.value):
        name = names.raw[32 * k:32 * (k + 1)].split(b"\0", 1)[0].decode()
        out[name] = (int(counts[k]), float(ms[k]))
    return out
