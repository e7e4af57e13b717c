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


def max_rel_inf(a, b):
    """max |a - b| over the group, relative to max |b| of the group."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    if a.size == 0:
        return 0.0
    den = np.abs(b).max()
    d = np.abs(a - b).max()
    return float(d / den) if den > 0 else float(d)


def assert_grad_close(got, ref, name, rel=1e-3, elem=1e-3):
    """Gradient parity of one parameter group: relative L2 <= rel and, per
    element, |got - ref| <= elem * max|ref| (a few wrong elements cannot hide
    inside the norm of the group)."""
    r, e = rel_l2(got, ref), max_rel_inf(got, ref)
    assert r <= rel, f"{name}: relative L2 {r:.2e} > {rel:.0e}"
    assert e <= elem, f"{name}: max element error {e:.2e} of max|ref| > {elem:.0e}"
    return r, e


def assert_sorted_match(keys, vals, rkeys, rvals, fragile):
    """Sorted instances bit for bit against the oracle's; the instances of
    fragile Gaussians (whose FP64 rect is within rounding of a tile edge, so
    that FP32 and FP64 may bin them differently) are excluded from both
    sides, every other instance must be equal and in the same order."""
    fragile = np.asarray(fragile, np.uint32)
    if len(fragile) == 0:
        assert len(keys) == len(rkeys)
        assert np.array_equal(keys, rkeys)
        assert np.array_equal(vals, rvals)
        return
    keep_g = ~np.isin(vals, fragile)
    keep_r = ~np.isin(rvals, fragile)
    assert np.array_equal(keys[keep_g], rkeys[keep_r])
    assert np.array_equal(vals[keep_g], rvals[keep_r])
