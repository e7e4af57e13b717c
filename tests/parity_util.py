"""Helpers shared by the GPU parity tests: identical float32 inputs for the
HIP path and the oracle, and the comparison rules.

Inputs come from paper_2410_08743_amd.synthetic (seeded); cameras are
rounded to float32 first so that the oracle sees exactly the intrinsics the
GPU library receives.
"""
import numpy as np

from paper_2410_08743_amd import synthetic as S


def f32_camera(cam):
    f = lambda x: float(np.float32(x))
    return S.Camera(cam.width, cam.height, f(cam.fx), f(cam.fy), f(cam.cx), f(cam.cy), cam.roi,
                    tuple(f(b) for b in cam.bg))


def rel_l2(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def random_case(seed, degree, W, H, n, roi=None, depth=(0.3, 6.0), lateral=1.4, bg=(0.1, 0.2, 0.05)):
    cam = S.Camera(W, H, W * 0.9 + 0.3, W * 0.9 - 0.2, W / 2 + 0.25, H / 2 - 0.4, roi=roi, bg=bg)
    cam = f32_camera(cam)
    sc = S.random_scene(seed, n, degree, cam, depth=depth, lateral=lateral)
    pose = S.random_pose_near_identity(seed, 4.0, 0.1)
    return sc, cam, pose


def unpack_rect(r):
    r = np.asarray(r, dtype=np.int64).reshape(-1, 2)
    lo, hi = r[:, 0], r[:, 1]
    return np.stack([lo & 0xFFFF, lo >> 16, hi & 0xFFFF, hi >> 16], axis=1)
