"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws numbers: Gaussian sets, cameras, poses and pose
perturbations.  It holds none of the rendering method's arithmetic and
imports nothing else from this package, so the HIP path and the CPU oracle can
both take their inputs from it.

The paper evaluates on LLFF, Replica and Tanks and Temples scenes with trained
models (Sec. IV); none of those are used.  The scenes below stand in for their
shapes: forward-facing slabs of Gaussians in front of a pinhole camera at the
image sizes and focal lengths of the workload definitions.

Poses are world-to-camera [R | t] (3 x 4); camera axes are x right, y down,
z forward.  Quaternions are (w, x, y, z).
"""
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np
from scipy.spatial.transform import Rotation

SH_C0 = 0.28209479177387814  # degree-0 basis constant 1 / (2 sqrt(pi))


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    roi: Optional[Tuple[int, int, int, int]] = None   # (x, y, w, h); None = full image
    bg: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    def region(self):
        return self.roi if self.roi is not None else (0, 0, self.width, self.height)

    def with_roi(self, roi):
        return Camera(self.width, self.height, self.fx, self.fy, self.cx, self.cy,
                      tuple(int(r) for r in roi), self.bg)


@dataclass
class GaussianSet:
    means: np.ndarray        # [n, 3] float32
    scales: np.ndarray       # [n, 3] float32, activated (> 0)
    quats: np.ndarray        # [n, 4] float32, (w, x, y, z), not normalised
    opacities: np.ndarray    # [n]    float32, activated (0, 1)
    sh: np.ndarray           # [n, S, 3] float32
    sh_degree: int = 0

    @property
    def n(self):
        return int(self.means.shape[0])

    def subset(self, idx):
        return GaussianSet(self.means[idx], self.scales[idx], self.quats[idx],
                           self.opacities[idx], self.sh[idx], self.sh_degree)


@dataclass
class Workload:
    name: str
    scene: GaussianSet
    camera: Camera
    pose: np.ndarray                       # ground-truth world->camera pose [3, 4] float32
    init_pose: Optional[np.ndarray] = None  # perturbed starting pose [3, 4] float32
    extra: dict = field(default_factory=dict)


def rng_for(seed: int, stream: int = 0) -> np.random.Generator:
    """Independent sub-streams of one seed."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream])))


def random_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def colour_sh(rng, n, degree, base=None, higher_std=0.2):
    """SH coefficients whose degree-0 term reproduces a base colour U(0,1)
    (colour = SH_C0 * f_dc + 1/2) and whose higher terms are N(0, std^2)."""
    S = (degree + 1) ** 2
    sh = np.zeros((n, S, 3), dtype=np.float64)
    if base is None:
        base = rng.uniform(0.0, 1.0, size=(n, 3))
    sh[:, 0, :] = (base - 0.5) / SH_C0
    if S > 1:
        sh[:, 1:, :] = rng.normal(0.0, higher_std, size=(n, S - 1, 3))
    return sh.astype(np.float32)


def look_at_pose(center, target, up=(0.0, -1.0, 0.0)):
    """World->camera pose of a camera at `center` looking at `target` with
    image y pointing along -up."""
    center = np.asarray(center, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - center
    fwd /= np.linalg.norm(fwd)
    upv = np.asarray(up, dtype=np.float64)
    right = np.cross(upv, fwd)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])       # rows: camera axes in world coordinates
    t = -R @ center
    return np.concatenate([R, t[:, None]], axis=1)


def camera_center(pose):
    pose = np.asarray(pose, dtype=np.float64)
    return -pose[:, :3].T @ pose[:, 3]


def perturb_pose(pose, rot_deg, trans, rng):
    """Rotates the camera by exactly rot_deg about a uniformly random axis
    (applied on the world->camera side) and moves its centre by exactly
    `trans` in a uniformly random direction."""
    pose = np.asarray(pose, dtype=np.float64)
    axis = rng.standard_normal(3)
    axis /= np.linalg.norm(axis)
    dirn = rng.standard_normal(3)
    dirn /= np.linalg.norm(dirn)
    R0 = pose[:, :3]
    c0 = camera_center(pose)
    R1 = Rotation.from_rotvec(np.deg2rad(rot_deg) * axis).as_matrix() @ R0
    c1 = c0 + trans * dirn
    t1 = -R1 @ c1
    return np.concatenate([R1, t1[:, None]], axis=1)


def pose_error(pose_est, pose_gt):
    """(rotation error in degrees, camera-centre distance)."""
    Re = np.asarray(pose_est, dtype=np.float64)[:, :3]
    Rg = np.asarray(pose_gt, dtype=np.float64)[:, :3]
    ang = np.rad2deg(Rotation.from_matrix(Re @ Rg.T).magnitude())
    dist = np.linalg.norm(camera_center(pose_est) - camera_center(pose_gt))
    return float(ang), float(dist)


def frustum_slab(rng, n, cam, z_range, lateral=1.1):
    """Means uniform in the volume of the camera frustum between two depths
    (camera at the origin looking along +z): pdf of z proportional to z^2."""
    z0, z1 = z_range
    z = np.cbrt(z0 ** 3 + rng.uniform(0.0, 1.0, n) * (z1 ** 3 - z0 ** 3))
    hx = lateral * (cam.width / 2.0) / cam.fx
    hy = lateral * (cam.height / 2.0) / cam.fy
    x = rng.uniform(-hx, hx, n) * z
    y = rng.uniform(-hy, hy, n) * z
    return np.stack([x, y, z], axis=1)


# --------------------------------------------------------------------------
# Workloads.  Seeds are 1000 + workload number; streams split scene / poses.
# --------------------------------------------------------------------------

def tiny(seed=1001):
    """1000 Gaussians, means U[-1,1]^3, log-scales U[log .01, log .1], random
    unit quaternions, opacity U(.1,.9), SH degree 0 colour U(0,1); pinhole
    camera at (0,0,-4) looking +z, 128x128, fx=fy=128.  Target pose: 2 deg
    rotation and 0.05 translation away."""
    rng = rng_for(seed, 0)
    n = 1000
    means = rng.uniform(-1.0, 1.0, (n, 3)).astype(np.float32)
    scales = np.exp(rng.uniform(np.log(0.01), np.log(0.1), (n, 3))).astype(np.float32)
    quats = random_quats(rng, n)
    opac = rng.uniform(0.1, 0.9, n).astype(np.float32)
    sh = colour_sh(rng, n, 0)
    cam = Camera(128, 128, 128.0, 128.0, 64.0, 64.0)
    pose = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 4.0]], dtype=np.float64)
    target = perturb_pose(pose, 2.0, 0.05, rng_for(seed, 1))
    return Workload("tiny-1k-128x128-sh0", GaussianSet(means, scales, quats, opac, sh, 0), cam,
                    pose.astype(np.float32), target.astype(np.float32))


def single_view(seed=1002, n=200_000):
    """Forward-facing slab scene for single-view pose estimation: 200k
    Gaussians in the frustum between depth 1.5 and 8, SH degree 3 (DC from a
    U(0,1) colour, higher terms N(0, 0.2^2)), 1008x756 image, fx=fy=815.
    Initial pose error exactly 5 deg / 0.1."""
    rng = rng_for(seed, 0)
    cam = Camera(1008, 756, 815.0, 815.0, 504.0, 378.0)
    means = frustum_slab(rng, n, cam, (1.5, 8.0)).astype(np.float32)
    scales = np.exp(rng.uniform(np.log(0.01), np.log(0.05), (n, 3))).astype(np.float32)
    quats = random_quats(rng, n)
    opac = rng.uniform(0.1, 0.9, n).astype(np.float32)
    sh = colour_sh(rng, n, 3)
    pose = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    init = perturb_pose(pose, 5.0, 0.1, rng_for(seed, 1))
    return Workload("pose-200k-1008x756-sh3", GaussianSet(means, scales, quats, opac, sh, 3), cam,
                    pose.astype(np.float32), init.astype(np.float32))


def arc_views(n_views=20, radius=4.75, half_angle_deg=10.0):
    """Ground-truth cameras on a forward-facing arc around (0, 0, radius),
    each looking at that point."""
    target = np.array([0.0, 0.0, radius])
    poses = []
    for th in np.deg2rad(np.linspace(-half_angle_deg, half_angle_deg, n_views)):
        center = target + radius * np.array([np.sin(th), 0.0, -np.cos(th)])
        poses.append(look_at_pose(center, target))
    return poses


def joint(seed=1003, n=1_000_000, n_views=20):
    """1M Gaussians in the slab (log-scales U[log .005, log .03]), SH degree 3,
    20 views of 1008x756 on a forward-facing arc, each with 3 deg / 0.05 of
    pose noise."""
    rng = rng_for(seed, 0)
    cam = Camera(1008, 756, 815.0, 815.0, 504.0, 378.0)
    means = frustum_slab(rng, n, cam, (1.5, 8.0)).astype(np.float32)
    scales = np.exp(rng.uniform(np.log(0.005), np.log(0.03), (n, 3))).astype(np.float32)
    quats = random_quats(rng, n)
    opac = rng.uniform(0.1, 0.9, n).astype(np.float32)
    sh = colour_sh(rng, n, 3)
    gt = arc_views(n_views)
    prng = rng_for(seed, 1)
    noisy = [perturb_pose(p, 3.0, 0.05, prng) for p in gt]
    wl = Workload("joint-1M-4x1008x756-sh3", GaussianSet(means, scales, quats, opac, sh, 3), cam,
                  gt[0].astype(np.float32), noisy[0].astype(np.float32))
    wl.extra["gt_poses"] = np.stack(gt).astype(np.float32)
    wl.extra["noisy_poses"] = np.stack(noisy).astype(np.float32)
    return wl


def room(seed=1004, n=500_000, n_frames=100):
    """Synthetic indoor scene for sequential tracking: a 6 x 3 x 5 box room
    (x in [-3, 3], y in [-1.5, 1.5] with y down, z in [-2.5, 2.5]); 80 % of
    the means on the six walls (normal jitter N(0, 0.01^2), scale along the
    wall normal x0.1), 20 % inside 10 random boxes; log-scales
    U[log .01, log .04], opacities U(.3, .95), SH degree 3 with a smoothly
    varying base colour and higher terms N(0, 0.05^2).  Camera 1200x680, fx = fy = 600, principal point at
    the centre.  Trajectory: a smooth random walk of n_frames poses inside
    the room, about 0.05 units and 1.5 degrees of yaw per frame, looking
    roughly along the room's long axis."""
    rng = rng_for(seed, 0)
    half = np.array([3.0, 1.5, 2.5])
    n_wall = int(0.8 * n)
    face = rng.integers(0, 6, n_wall)
    axis = face // 2
    sign = np.where(face % 2 == 0, -1.0, 1.0)
    means = rng.uniform(-1.0, 1.0, (n, 3)) * half
    idx = np.arange(n_wall)
    means[idx, axis] = sign * half[axis] + rng.normal(0.0, 0.01, n_wall)
    centres = rng.uniform(-1.0, 1.0, (10, 3)) * (half - 0.6)
    sizes = rng.uniform(0.15, 0.5, (10, 3))
    which = rng.integers(0, 10, n - n_wall)
    means[n_wall:] = centres[which] + rng.uniform(-1.0, 1.0, (n - n_wall, 3)) * sizes[which]
    scales = np.exp(rng.uniform(np.log(0.01), np.log(0.04), (n, 3)))
    scales[idx, axis] *= 0.1
    # wall Gaussians keep the identity rotation, so their thin axis is the
    # wall normal; the others are turned at random
    quats = np.zeros((n, 4), dtype=np.float32)
    quats[:, 0] = 1.0
    quats[n_wall:] = random_quats(rng, n - n_wall)
    opac = rng.uniform(0.3, 0.95, n).astype(np.float32)
    # colour varies smoothly over the room (a sum of plane waves of 0.3-1.5
    # wavelength per channel, plus small per-Gaussian jitter), like painted
    # walls and furniture: per-Gaussian white-noise colour would leave frame
    # to frame tracking no basin of attraction at these motions
    base = np.full((n, 3), 0.5)
    for ch in range(3):
        for _ in range(4):
            kvec = rng.normal(0.0, 1.0, 3)
            kvec *= 2.0 * np.pi / (rng.uniform(0.3, 1.5) * np.linalg.norm(kvec))
            base[:, ch] += 0.12 * np.sin(means @ kvec + rng.uniform(0.0, 2.0 * np.pi))
    base = np.clip(base + rng.normal(0.0, 0.03, (n, 3)), 0.0, 1.0)
    sh = colour_sh(rng, n, 3, base=base, higher_std=0.05)
    cam = Camera(1200, 680, 600.0, 600.0, 600.0, 340.0)
    trng = rng_for(seed, 1)
    pos = np.array([0.0, 0.2, -1.6])
    yaw = 0.0
    vel = np.zeros(3)
    poses = []
    for _ in range(n_frames):
        vel = 0.7 * vel + 0.3 * trng.normal(0.0, 0.05, 3) * np.array([1.0, 0.2, 1.0])
        vel *= 0.05 / max(np.linalg.norm(vel), 1e-9)
        pos = np.clip(pos + vel, -half + 0.8, half - 0.8)
        yaw += np.deg2rad(trng.normal(0.0, 1.5))
        yaw = float(np.clip(yaw, -np.deg2rad(30.0), np.deg2rad(30.0)))
        fwd = np.array([np.sin(yaw), 0.0, np.cos(yaw)])
        poses.append(look_at_pose(pos, pos + fwd))
    wl = Workload("track-500k-1200x680-sh3", GaussianSet(means.astype(np.float32),
                  scales.astype(np.float32), quats, opac, sh, 3), cam,
                  poses[0].astype(np.float32), None)
    wl.extra["trajectory"] = np.stack(poses).astype(np.float32)
    return wl


def box_depth(cam, pose, half=(3.0, 1.5, 2.5)):
    """Camera-frame depth [H, W] of the walls of the axis-aligned box
    [-half, half] seen from inside it (rays through pixel centres): the
    stand-in for a monocular depth estimate of a room frame (it knows the
    walls, not the objects in the room)."""
    pose = np.asarray(pose, dtype=np.float64)
    R, t = pose[:, :3], pose[:, 3]
    o = -R.T @ t
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    dc = np.stack([(xs + 0.5 - cam.cx) / cam.fx, (ys + 0.5 - cam.cy) / cam.fy,
                   np.ones(xs.shape)], axis=-1)
    dw = dc @ R                       # R^T d per pixel
    h = np.asarray(half, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        tt = np.where(dw > 0, (h - o) / dw, np.where(dw < 0, (-h - o) / dw, np.inf))
    return tt.min(axis=-1).astype(np.float32)


def depth_coloured(scene, pose):
    """The scene with every Gaussian's colour set to its camera-frame depth
    under `pose` (SH degree-0 term only): a render of it divided by its
    accumulated opacity is the expected depth map of the view -- the
    stand-in for a monocular depth estimate of a frame."""
    pose = np.asarray(pose, dtype=np.float64)
    z = (np.asarray(scene.means, dtype=np.float64) @ pose[:, :3].T + pose[:, 3])[:, 2]
    sh = np.zeros((scene.n, 1, 3), dtype=np.float32)
    sh[:, 0, :] = ((z - 0.5) / 0.28209479177387814)[:, None]
    return GaussianSet(scene.means, scene.scales, scene.quats, scene.opacities, sh, 0)


REQUEST_SIZES = ((320, 240), (640, 480), (1008, 756))


def serving_requests(seed=1005, n_requests=64, sizes=REQUEST_SIZES, radius=4.75,
                     half_angle_deg=10.0):
    """Pose-estimation requests against the joint scene (served resident):
    image size uniform over `sizes`, same field of view as the 1008x756
    camera (fx = fy = 815 W / 1008, principal point at the centre); ground
    truth a uniform point of the arc of `joint` with the camera centre
    jittered by U(-0.05, 0.05) per axis, still looking at the arc's centre;
    starting pose the ground truth turned by U(1, 5) degrees and moved by
    U(0.02, 0.1).  `gap` is a unit-rate exponential inter-arrival time (scale
    by 1/rate for Poisson arrivals at that rate)."""
    rng = rng_for(seed, 0)
    target = np.array([0.0, 0.0, radius])
    out = []
    for k in range(n_requests):
        W, H = sizes[int(rng.integers(len(sizes)))]
        f = 815.0 * W / 1008.0
        cam = Camera(W, H, f, f, W / 2.0, H / 2.0)
        th = np.deg2rad(rng.uniform(-half_angle_deg, half_angle_deg))
        center = target + radius * np.array([np.sin(th), 0.0, -np.cos(th)])
        center = center + rng.uniform(-0.05, 0.05, 3)
        gt = look_at_pose(center, target)
        init = perturb_pose(gt, rng.uniform(1.0, 5.0), rng.uniform(0.02, 0.1), rng_for(seed, 1 + k))
        out.append({"rid": k, "camera": cam, "gt_pose": gt.astype(np.float32),
                    "init_pose": init.astype(np.float32), "gap": float(rng.exponential(1.0))})
    return out


def random_scene(seed, n, sh_degree, cam, depth=(1.0, 6.0), log_scale=(np.log(0.02), np.log(0.3)),
                 opacity=(0.05, 0.99), lateral=1.3, higher_std=0.3):
    """Small random scenes for property and parity tests: Gaussians in (and
    slightly beyond) the frustum of a camera at the origin."""
    rng = rng_for(seed, 0)
    means = frustum_slab(rng, n, cam, depth, lateral).astype(np.float32)
    scales = np.exp(rng.uniform(log_scale[0], log_scale[1], (n, 3))).astype(np.float32)
    quats = random_quats(rng, n)
    opac = rng.uniform(opacity[0], opacity[1], n).astype(np.float32)
    sh = colour_sh(rng, n, sh_degree, higher_std=higher_std)
    return GaussianSet(means, scales, quats, opac, sh, sh_degree)


def identity_pose():
    return np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)


def random_pose_near_identity(seed, rot_deg=3.0, trans=0.1):
    return perturb_pose(identity_pose(), rot_deg, trans, rng_for(seed, 7)).astype(np.float32)


def upstream(seed, shape):
    """A fixed random upstream gradient dL/dimage."""
    return rng_for(seed, 3).standard_normal(shape).astype(np.float32)
