"""FP64 CPU oracle of the pose-differentiable Gaussian splatting rasterizer.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this package.  It shares no code with
the HIP library and imports nothing from the product package: scenes and
cameras are accepted by duck typing (attributes ``means, scales, quats,
opacities, sh, sh_degree`` and ``width, height, fx, fy, cx, cy, roi, bg``).

Every array crosses the C boundary as float64 (FP32 inputs widen exactly).
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

__all__ = [
    "load", "SPLAT_DTYPE", "TRACE_DTYPE", "sh_basis", "quat_to_rotmat",
    "se3_exp", "se3_retract", "preprocess", "count_instances", "bin_sort",
    "tile_ranges", "render", "render_brute", "pixel_trace", "backward", "l1",
    "masked_l1", "pose_adam", "TILE", "tiles_of", "max_threads", "set_threads",
]

TILE = 16

SPLAT_DTYPE = np.dtype([
    ("u", "f8"), ("v", "f8"), ("cov", "f8", 3), ("conic", "f8", 3),
    ("color", "f8", 3), ("p", "f8", 3), ("opacity", "f8"),
    ("depth_key", "f4"), ("radius", "i4"), ("rect", "i4", 4),
    ("rendered", "i4"), ("fragile", "i4"), ("color_clamped", "i4", 3),
    ("jclamp", "i4", 2),
], align=True)

TRACE_DTYPE = np.dtype([
    ("gaussian", "i4"), ("position", "i4"), ("blended", "i4"),
    ("alpha_clamped", "i4"), ("power", "f8"), ("alpha", "f8"),
    ("T_before", "f8"),
], align=True)


class _View(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("roi_x", ctypes.c_int32), ("roi_y", ctypes.c_int32),
                ("roi_w", ctypes.c_int32), ("roi_h", ctypes.c_int32),
                ("bg", ctypes.c_double * 3)]


class _Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacities", ctypes.c_void_p),
                ("sh", ctypes.c_void_p)]


class _Grads(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("means", "scales", "quats", "opacities", "sh", "splat2d",
                 "pose", "pose_parts")]


_lib = None


def load():
    """Loads liboracle.so, building it first if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    lib.gso_max_threads.restype = ctypes.c_int
    lib.gso_set_threads.argtypes = [ctypes.c_int]
    lib.gso_sh_basis.argtypes = [ctypes.c_int, P, P, P]
    lib.gso_quat_to_rotmat.argtypes = [P, P]
    lib.gso_se3_exp.argtypes = [P, P]
    lib.gso_se3_retract.argtypes = [P, P]
    lib.gso_preprocess.argtypes = [P, P, P, P]
    lib.gso_count_instances.argtypes = [ctypes.c_int32, ctypes.c_int64, P]
    lib.gso_count_instances.restype = ctypes.c_int64
    lib.gso_bin_sort.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P,
                                 ctypes.c_int64, P, P]
    lib.gso_bin_sort.restype = ctypes.c_int64
    lib.gso_tile_ranges.argtypes = [ctypes.c_int64, P, ctypes.c_int64, P]
    lib.gso_render.argtypes = [P, P, P, P, P, P, P, P]
    lib.gso_render_brute.argtypes = [P, P, P, P, P]
    lib.gso_pixel_trace.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_int32, P,
                                    ctypes.c_int32]
    lib.gso_backward.argtypes = [P, P, P, P, P]
    lib.gso_l1.argtypes = [ctypes.c_int64, P, P, P]
    lib.gso_l1.restype = ctypes.c_double
    lib.gso_masked_l1.argtypes = [ctypes.c_int64, P, P, P, P]
    lib.gso_masked_l1.restype = ctypes.c_double
    lib.gso_pose_adam.argtypes = [P, P, P, P, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


class _Scene:
    """Keeps float64 copies alive while the C structure points at them."""

    def __init__(self, scene):
        n = int(np.asarray(scene.means).shape[0])
        self.n = n
        self.sh_degree = int(scene.sh_degree)
        S = (self.sh_degree + 1) ** 2
        self.means = _f64(scene.means, (n, 3))
        self.scales = _f64(scene.scales, (n, 3))
        self.quats = _f64(scene.quats, (n, 4))
        self.opacities = _f64(scene.opacities, (n,))
        self.sh = _f64(scene.sh, (n, S, 3))
        self.c = _Gaussians(n, self.sh_degree, _ptr(self.means), _ptr(self.scales),
                            _ptr(self.quats), _ptr(self.opacities), _ptr(self.sh))


def _view(cam):
    roi = getattr(cam, "roi", None) or (0, 0, cam.width, cam.height)
    bg = getattr(cam, "bg", None)
    bg = (0.0, 0.0, 0.0) if bg is None else tuple(float(b) for b in bg)
    return _View(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy),
                 float(cam.cx), float(cam.cy), int(roi[0]), int(roi[1]),
                 int(roi[2]), int(roi[3]), (ctypes.c_double * 3)(*bg))


def _pose(pose):
    return _f64(pose, (12,))


def max_threads():
    return int(load().gso_max_threads())


def set_threads(n):
    """Number of OpenMP threads of later oracle calls."""
    load().gso_set_threads(int(n))


def tiles_of(cam):
    roi = getattr(cam, "roi", None) or (0, 0, cam.width, cam.height)
    return (roi[2] + TILE - 1) // TILE, (roi[3] + TILE - 1) // TILE


def sh_basis(degree, d, with_grad=False):
    lib = load()
    S = (degree + 1) ** 2
    d = _f64(d, (3,))
    Y = np.zeros(S)
    G = np.zeros((S, 3)) if with_grad else None
    lib.gso_sh_basis(degree, _ptr(d), _ptr(Y), _ptr(G))
    return (Y, G) if with_grad else Y


def quat_to_rotmat(q):
    lib = load()
    q = _f64(q, (4,))
    R = np.zeros(9)
    lib.gso_quat_to_rotmat(_ptr(q), _ptr(R))
    return R.reshape(3, 3)


def se3_exp(tau):
    lib = load()
    tau = _f64(tau, (6,))
    T = np.zeros(12)
    lib.gso_se3_exp(_ptr(tau), _ptr(T))
    return T.reshape(3, 4)


def se3_retract(delta, pose):
    lib = load()
    delta = _f64(delta, (6,))
    T = _f64(pose, (12,)).copy()
    lib.gso_se3_retract(_ptr(delta), _ptr(T))
    return T.reshape(3, 4)


def preprocess(scene, cam, pose):
    lib = load()
    sc = _Scene(scene)
    out = np.zeros(sc.n, dtype=SPLAT_DTYPE)
    v = _view(cam)
    p = _pose(pose)
    rc = lib.gso_preprocess(ctypes.byref(sc.c), ctypes.byref(v), _ptr(p), _ptr(out))
    if rc != 0:
        raise ValueError("gso_preprocess rejected its arguments")
    return out


def count_instances(splat_list):
    lib = load()
    arrs = [np.ascontiguousarray(s) for s in splat_list]
    ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    return lib.gso_count_instances(len(arrs), len(arrs[0]), ptrs)


def bin_sort(splat_list, tiles):
    """Sorted (keys, values) over the views; tiles = [(gw, gh), ...]."""
    lib = load()
    arrs = [np.ascontiguousarray(s) for s in splat_list]
    ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    M = lib.gso_count_instances(len(arrs), len(arrs[0]), ptrs)
    keys = np.zeros(max(M, 1), dtype=np.uint64)
    vals = np.zeros(max(M, 1), dtype=np.uint32)
    tx = np.array([t[0] for t in tiles], dtype=np.int32)
    ty = np.array([t[1] for t in tiles], dtype=np.int32)
    got = lib.gso_bin_sort(len(arrs), len(arrs[0]), ptrs, _ptr(tx), _ptr(ty), M,
                           _ptr(keys), _ptr(vals))
    if got != M:
        raise RuntimeError("gso_bin_sort failed")
    return keys[:M], vals[:M]


def tile_ranges(keys, ntiles):
    lib = load()
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.zeros((ntiles, 2), dtype=np.uint32)
    lib.gso_tile_ranges(len(keys), _ptr(keys), ntiles, _ptr(out))
    return out


def _roi_shape(cam):
    roi = getattr(cam, "roi", None) or (0, 0, cam.width, cam.height)
    return int(roi[3]), int(roi[2])


def render(scene, cam, pose, signature=False):
    lib = load()
    sc = _Scene(scene)
    v = _view(cam)
    p = _pose(pose)
    h, w = _roi_shape(cam)
    image = np.zeros((3, h, w))
    T = np.zeros((h, w))
    nc = np.zeros((h, w), dtype=np.int32)
    strad = np.zeros((h, w), dtype=np.uint8)
    sig = np.zeros(1, dtype=np.uint64) if signature else None
    rc = lib.gso_render(ctypes.byref(sc.c), ctypes.byref(v), _ptr(p), _ptr(image),
                        _ptr(T), _ptr(nc), _ptr(strad), _ptr(sig))
    if rc != 0:
        raise ValueError("gso_render rejected its arguments")
    out = {"image": image, "T_final": T, "n_contrib": nc, "straddle": strad.astype(bool)}
    if signature:
        out["signature"] = int(sig[0])
    return out


def render_brute(scene, cam, pose):
    lib = load()
    sc = _Scene(scene)
    v = _view(cam)
    p = _pose(pose)
    h, w = _roi_shape(cam)
    image = np.zeros((3, h, w))
    T = np.zeros((h, w))
    rc = lib.gso_render_brute(ctypes.byref(sc.c), ctypes.byref(v), _ptr(p), _ptr(image), _ptr(T))
    if rc != 0:
        raise ValueError("gso_render_brute rejected its arguments")
    return {"image": image, "T_final": T}


def pixel_trace(scene, cam, pose, px, py, max_entries=100000):
    lib = load()
    sc = _Scene(scene)
    v = _view(cam)
    p = _pose(pose)
    out = np.zeros(max_entries, dtype=TRACE_DTYPE)
    nt = lib.gso_pixel_trace(ctypes.byref(sc.c), ctypes.byref(v), _ptr(p), int(px), int(py),
                             _ptr(out), max_entries)
    if nt < 0:
        raise ValueError("gso_pixel_trace rejected its arguments")
    return out[:nt]


def backward(scene, cam, pose, dl_dimage):
    lib = load()
    sc = _Scene(scene)
    v = _view(cam)
    p = _pose(pose)
    h, w = _roi_shape(cam)
    G = _f64(dl_dimage, (3, h, w))
    n, S = sc.n, (sc.sh_degree + 1) ** 2
    out = {
        "means": np.zeros((n, 3)), "scales": np.zeros((n, 3)), "quats": np.zeros((n, 4)),
        "opacities": np.zeros(n), "sh": np.zeros((n, S, 3)), "splat2d": np.zeros((n, 9)),
        "pose": np.zeros(6), "pose_parts": np.zeros(18),
    }
    g = _Grads(*[_ptr(out[k]) for k in ("means", "scales", "quats", "opacities", "sh",
                                         "splat2d", "pose", "pose_parts")])
    rc = lib.gso_backward(ctypes.byref(sc.c), ctypes.byref(v), _ptr(p), _ptr(G), ctypes.byref(g))
    if rc != 0:
        raise ValueError("gso_backward rejected its arguments")
    return out


def l1(a, b):
    lib = load()
    a = _f64(a).ravel()
    b = _f64(b).ravel()
    grad = np.zeros_like(a)
    val = lib.gso_l1(a.size, _ptr(a), _ptr(b), _ptr(grad))
    return val, grad


def masked_l1(a, b, T_final):
    lib = load()
    a = _f64(a)
    b = _f64(b)
    T = _f64(T_final)
    grad = np.zeros_like(a)
    val = lib.gso_masked_l1(T.size, _ptr(a), _ptr(b), _ptr(T), _ptr(grad))
    return val, grad


def pose_adam(pose, m, v, g, k, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Returns (new_pose, m, v, delta) after one tangent Adam step."""
    lib = load()
    T = _f64(pose, (12,)).copy()
    m = _f64(m, (6,)).copy()
    v = _f64(v, (6,)).copy()
    g = _f64(g, (6,))
    delta = np.zeros(6)
    lib.gso_pose_adam(_ptr(T), _ptr(m), _ptr(v), _ptr(g), int(k), float(lr), float(beta1),
                      float(beta2), float(eps), _ptr(delta))
    return T.reshape(3, 4), m, v, delta
