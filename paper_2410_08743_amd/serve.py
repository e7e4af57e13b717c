"""Continuous-batching pose-estimation server over a resident Gaussian scene.

A request is a target image with its intrinsics and a starting pose; solving
it means `iters` tangent-space Adam iterations on the L1 loss (Sec. III-B,
the pose-estimation use of Eq. (5)-(13)).  The server keeps the scene on the
device and runs every request that is in flight in ONE launch per iteration:
one view per request, each of its own size, through the library's batched
render-with-L1 (one pass), backward and Adam calls.  Requests that arrive while others
are running join at the next iteration boundary when a batch slot and enough
of the HBM budget are free, and leave when their last iteration is done, so
work from different requests overlaps on the device (continuous batching).

Everything a request computes depends on its own view only (per-view
projection, per-tile lists, per-view loss normalisation, per-view pose
reduction in a fixed order, per-view Adam state), so its result is the same,
bit for bit, alone or in any mix.

The host thread only schedules: it builds each iteration's view table,
enqueues the library calls on one stream and keeps at most `depth`
iterations in flight; per-iteration overflow flags come back through pinned
memory.  An iteration whose render ran out of instance capacity leaves every
pose of the launch unchanged (the Adam step is guarded on the device); the
host repeats it for the requests concerned with a larger capacity.
"""
import ctypes
import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _native as N
from . import render as R


@dataclass
class PoseRequest:
    camera: object                 # intrinsics of the request's image (synthetic.Camera)
    target: torch.Tensor           # [3, h, w] float32 on the server's device
    init_pose: torch.Tensor        # [3, 4] float32 on the device, world->camera
    arrival: float = 0.0           # seconds after run() starts, or an iteration index
    rid: int = 0


@dataclass
class PoseResult:
    rid: int
    pose: np.ndarray               # [3, 4] final world->camera pose
    arrival: float
    admitted: float
    completed: float
    latency: float                 # completed - arrival
    iterations: int                # applied Adam iterations
    batch_sizes: List[int] = field(default_factory=list)


class _Live:
    """Book-keeping of one admitted request."""

    def __init__(self, req, dl, nbytes, admitted):
        self.req = req
        self.dl = dl
        self.nbytes = nbytes
        self.admitted = admitted
        self.enqueued = 0            # iterations enqueued and not known to be void
        self.retired_at = None       # iteration of its last enqueue, while awaiting confirmation
        self.saved = None            # device state copied out at retirement
        self.batch_sizes = []


class PoseServer:
    """Serves pose-estimation requests against one resident scene `g`."""

    def __init__(self, g: R.GaussianParams, iters: int = 50, lr=(1e-2, 1e-4), betas=(0.9, 0.999),
                 eps: float = 1e-8, max_batch: int = N.GSP_MAX_VIEWS, hbm_budget: int = 16 << 30,
                 depth: int = 2, margin: float = 1.25, device: Optional[int] = None):
        if not 1 <= max_batch <= N.GSP_MAX_VIEWS:
            raise ValueError(f"max_batch must be in 1..{N.GSP_MAX_VIEWS}")
        self.g = g
        self.iters = int(iters)
        self.lr = lr
        self.betas = betas
        self.eps = eps
        self.max_batch = int(max_batch)
        self.budget = int(hbm_budget)
        self.depth = max(1, int(depth))
        self.margin = float(margin)
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.dev = f"cuda:{self.device}"
        self.est = {}                # camera key -> instance estimate
        self.ws = None
        B = self.max_batch
        self.poses = torch.zeros((B, 3, 4), dtype=torch.float32, device=self.dev)
        self.m = torch.zeros((B, 6), dtype=torch.float32, device=self.dev)
        self.v = torch.zeros((B, 6), dtype=torch.float32, device=self.dev)
        self.steps = torch.zeros(B, dtype=torch.int32, device=self.dev)
        self.dpose = torch.zeros((B, 6), dtype=torch.float32, device=self.dev)
        self.adam = N.AdamParams(lr[0], lr[1], self.iters, betas[0], betas[1], eps, N.GSP_POSE_SE3)

    # -- sizing ------------------------------------------------------------
    @staticmethod
    def _key(cam):
        return (int(cam.width), int(cam.height), float(cam.fx), float(cam.fy), float(cam.cx),
                float(cam.cy), tuple(R.region(cam)))

    def calibrate(self, cam, pose: torch.Tensor):
        """Measures the instance count of one render of `cam` at `pose` and keeps
        it as the estimate for requests of that camera."""
        rast = R.Rasterizer(self.device)
        rast.forward(self.g, [cam], pose.reshape(1, 3, 4).contiguous())
        m, _ = rast.instances()
        self.est[self._key(cam)] = max(int(m), 1)
        return m

    def instances_estimate(self, cam):
        k = self._key(cam)
        if k not in self.est:
            raise KeyError("camera not calibrated; call calibrate() first")
        return int(self.est[k] * self.margin) + 4096

    def _ws_bytes(self, views, cap):
        sz = ctypes.c_size_t()
        N.check(N.lib().gsp_workspace_size(self.g.n, self.g.sh_degree, len(views), views, cap,
                                           ctypes.byref(sz)), "gsp_workspace_size")
        return sz.value

    def request_bytes(self, cam):
        """HBM a request holds while admitted: its share of the workspace (the
        per-view splat records, sorted instances, slots and per-pixel state,
        as one single-view workspace) plus its image gradient and target (the
        render and its L1 gradient are one pass; no image is kept)."""
        _, _, w, h = R.region(cam)
        ws1 = self._ws_bytes(N.view_array([cam]), self.instances_estimate(cam))
        return int(ws1 + 2 * 12 * w * h)

    # -- one iteration -----------------------------------------------------
    def _enqueue(self, running, it, pinned):
        L = N.lib()
        ctx = R.context(self.device)
        st = R._stream()
        V = len(running)
        cams = [x.req.camera for x in running]
        views = N.view_array(cams)
        cap = sum(self.instances_estimate(c) for c in cams)
        nbytes = self._ws_bytes(views, cap)
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = torch.zeros(int(nbytes * 1.25) + (1 << 20), dtype=torch.uint8, device=self.dev)
        gs = self.g.struct()
        dl = N.ptr_array([x.dl.data_ptr() for x in running])
        tgt = N.ptr_array([x.req.target.data_ptr() for x in running])
        wsp = ctypes.c_void_p(self.ws.data_ptr())
        poses = ctypes.c_void_p(self.poses.data_ptr())
        dpose = ctypes.c_void_p(self.dpose.data_ptr())
        N.check(L.gsp_render_fwd_l1(ctx, ctypes.byref(gs), V, views, poses, tgt, dl, None, None,
                                    wsp, nbytes, cap, st), "gsp_render_fwd_l1")
        # pose-only backward whose final pose reduction applies the Adam step
        # (bit-identical to gsp_render_bwd + gsp_pose_adam guarded by wsp)
        N.check(L.gsp_render_bwd_pose_step(ctx, ctypes.byref(gs), V, views, poses, dl, wsp, nbytes,
                                           cap, dpose, ctypes.c_void_p(self.m.data_ptr()),
                                           ctypes.c_void_p(self.v.data_ptr()),
                                           ctypes.c_void_p(self.steps.data_ptr()),
                                           ctypes.byref(self.adam), st), "gsp_render_bwd_pose_step")
        pinned.copy_(self.ws[:16], non_blocking=True)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        return ev, cap

    # -- state moves between batch positions -------------------------------
    def _save(self, p):
        return (self.poses[p].clone(), self.m[p].clone(), self.v[p].clone(), self.steps[p].clone())

    def _load(self, p, state):
        self.poses[p].copy_(state[0])
        self.m[p].copy_(state[1])
        self.v[p].copy_(state[2])
        self.steps[p].copy_(state[3])

    def _move(self, src, dst):
        self.poses[dst].copy_(self.poses[src])
        self.m[dst].copy_(self.m[src])
        self.v[dst].copy_(self.v[src])
        self.steps[dst].copy_(self.steps[src])

    # -- the serving loop --------------------------------------------------
    def run(self, requests: Sequence[PoseRequest], clock: str = "wall") -> List[PoseResult]:
        """Serves `requests` (arrival times in seconds from now with
        clock="wall", or iteration indices with clock="iterations") and
        returns one result per request, in request order."""
        if clock not in ("wall", "iterations"):
            raise ValueError("clock must be 'wall' or 'iterations'")
        for r in requests:
            if self._key(r.camera) not in self.est:
                self.calibrate(r.camera, r.init_pose)
            need = self.request_bytes(r.camera)
            if need > self.budget:
                raise ValueError(f"request {r.rid} needs {need} bytes, more than the HBM budget")
        order = sorted(range(len(requests)), key=lambda k: (requests[k].arrival, k))
        pending = deque(requests[k] for k in order)
        running: List[_Live] = []
        retired: List[_Live] = []
        inflight = deque()
        results = {}
        used = 0
        it = 0
        ring = [torch.zeros(16, dtype=torch.uint8).pin_memory() for _ in range(self.depth + 2)]
        torch.cuda.synchronize(self.device)
        start = torch.cuda.Event(enable_timing=True)
        start.record()
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0 if clock == "wall" else float(it)

        def admit(r):
            nonlocal used
            _, _, w, h = R.region(r.camera)
            x = _Live(r, torch.empty((3, h, w), dtype=torch.float32, device=self.dev),
                      self.request_bytes(r.camera), now())
            p = len(running)
            self.poses[p].copy_(r.init_pose)
            self.m[p].zero_()
            self.v[p].zero_()
            self.steps[p].zero_()
            running.append(x)
            used += x.nbytes

        def confirm(entry):
            nonlocal used
            k, ev, members, pin, cap = entry
            ev.synchronize()
            cnt = pin.view(torch.int32).numpy()
            overflow = int(cnt[2]) != 0
            if overflow:
                m_needed = (int(cnt[1]) << 32) | (int(cnt[0]) & 0xffffffff)
                grow = max(m_needed / max(cap, 1), 1.0) * 1.1
                for key in self.est:
                    self.est[key] = int(self.est[key] * grow) + 1
                for x in members:
                    x.enqueued -= 1
                    if x.retired_at is not None:     # its last iteration was void: run it again
                        x.retired_at = None
                        retired.remove(x)
                        p = len(running)
                        self._load(p, x.saved)
                        x.saved = None
                        running.append(x)
                return
            t_done = start.elapsed_time(ev) / 1e3 if clock == "wall" else float(k + 1)
            for x in members:
                if x.retired_at == k:
                    retired.remove(x)
                    used -= x.nbytes
                    pose = x.saved[0].cpu().numpy()
                    r = x.req
                    results[r.rid] = PoseResult(r.rid, pose, r.arrival, x.admitted, t_done,
                                                t_done - r.arrival, int(x.saved[3].item()),
                                                x.batch_sizes)
                    x.saved = None

        while pending or running or retired or inflight:
            t = now()
            # a retired request keeps its batch slot until its last iteration
            # is confirmed, so that a void last iteration can be re-run
            while (pending and pending[0].arrival <= t
                   and len(running) + len(retired) < self.max_batch
                   and used + self.request_bytes(pending[0].camera) <= self.budget):
                admit(pending.popleft())
            if running:
                members = list(running)
                pin = ring[it % len(ring)]
                ev, cap = self._enqueue(members, it, pin)
                for x in members:
                    x.enqueued += 1
                    x.batch_sizes.append(len(members))
                done = [p for p, x in enumerate(running) if x.enqueued >= self.iters]
                for p in sorted(done, reverse=True):
                    x = running[p]
                    x.saved = self._save(p)
                    x.retired_at = it
                    last = len(running) - 1
                    if p != last:
                        self._move(last, p)
                        running[p] = running[last]
                    running.pop()
                    retired.append(x)
                inflight.append((it, ev, members, pin, cap))
                it += 1
            while inflight and (len(inflight) > self.depth or not running
                                or inflight[0][1].query()):
                confirm(inflight.popleft())
            if not running and not inflight and pending:
                if clock == "wall":
                    wait = pending[0].arrival - now()
                    if wait > 0:
                        time.sleep(wait)
                else:
                    it = max(it, int(math.ceil(pending[0].arrival)))
        return [results[r.rid] for r in requests]


def serve_hypotheses(server: PoseServer, requests: Sequence[PoseRequest], clock: str = "wall"):
    """Multi-hypothesis pose estimation through the server: a request whose
    init_pose is [H, 3, 4] is served as H requests (one per start, sharing the
    target tensor) in the continuous batch, and its answer is the start whose
    final L1 is lowest (evaluated in renders of up to GSP_MAX_VIEWS results
    per launch).  Returns (one PoseResult per request -- the chosen
    hypothesis, completed when its last hypothesis completed -- and the index
    of the chosen start of each request)."""
    expanded, owner = [], []
    for q, r in enumerate(requests):
        inits = r.init_pose.reshape(-1, 3, 4)
        for h in range(inits.shape[0]):
            expanded.append(PoseRequest(r.camera, r.target, inits[h].contiguous(), r.arrival,
                                        len(expanded)))
            owner.append(q)
    res = server.run(expanded, clock=clock)
    losses = np.zeros(len(res))
    rast = R.Rasterizer(server.device)
    for a in range(0, len(res), N.GSP_MAX_VIEWS):
        idx = list(range(a, min(a + N.GSP_MAX_VIEWS, len(res))))
        cams = [expanded[k].camera for k in idx]
        poses = torch.tensor(np.stack([res[k].pose for k in idx]), device=server.dev)
        imgs, _ = rast.forward(server.g, cams, poses)
        loss, _ = R.loss_l1(cams, R.split_images(imgs, cams), [expanded[k].target for k in idx])
        losses[idx] = loss.cpu().numpy()
    out, chosen = [], []
    for q, r in enumerate(requests):
        ks = [k for k, o in enumerate(owner) if o == q]
        best = min(ks, key=lambda k: (losses[k], k))
        done = max(res[k].completed for k in ks)
        b = res[best]
        out.append(PoseResult(r.rid, b.pose, r.arrival, min(res[k].admitted for k in ks), done,
                              done - r.arrival, b.iterations, b.batch_sizes))
        chosen.append(best - ks[0])
    return out, chosen


def latency_stats(results: Sequence[PoseResult]):
    lat = np.array([r.latency for r in results], dtype=np.float64)
    span = max(r.completed for r in results) - min(r.arrival for r in results)
    return {"requests": len(results), "requests_per_s": len(results) / span if span > 0 else None,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_batch": float(np.mean([np.mean(r.batch_sizes) for r in results]))}


def fifo_latencies(arrivals: Sequence[float], service: Sequence[float]):
    """Completion times of a single first-come-first-served server with the
    given service times: c_k = max(a_k, c_{k-1}) + s_k."""
    c, out = 0.0, []
    for a, s in zip(arrivals, service):
        c = max(a, c) + s
        out.append(c)
    return out
