"""FP64 oracle of the scene initialisation used for relative pose estimation
between two frames (Sec. III-D): a depth map of frame t is unprojected
through the intrinsics into points, which become isotropic Gaussians with
the pixel's colour and, as scale, the mean distance to their three nearest
neighbours.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module.  numpy only; it imports
nothing from the product package and shares no code with the HIP library.
(The masked L1 of Eq. (20)-(21) is oracle.masked_l1.)

Readings where the paper is silent (each is also listed with the design
notes):
  * The pixel subset is a regular grid: pixels (stride i, stride j) of the
    region of interest, sampled at their centres.  The depth map holds the
    camera-frame z of each pixel; frame t's camera is the world frame.
  * Colour c of the pixel becomes the degree-0 SH coefficient
    (c - 1/2) / Y_0, Y_0 = 1 / (2 sqrt(pi)); higher coefficients are 0.
  * Opacity starts at a constant, 0.5 by default (high enough that
    overlapping neighbours reach the mask threshold of Eq. (20) where the
    depth map has surface); rotation is the identity quaternion.
  * Pixels whose depth is not a positive finite number still yield a
    Gaussian (at depth 1 on the pixel's ray, opacity sigmoid(-30), so that
    it never blends) and are nobody's neighbour.  Every point's scale is the
    mean over its three nearest valid neighbours; a point with fewer
    averages over those it has (scale 0.01 with none).
"""
import numpy as np

Y0 = 0.28209479177387814   # 1 / (2 sqrt(pi))
INVALID_LOGIT = -30.0
INVALID_SCALE = 0.01


def grid_shape(roi_w, roi_h, stride):
    return (roi_w + stride - 1) // stride, (roi_h + stride - 1) // stride


def knn3_mean_distance(points, valid=None):
    """The scale of Sec. III-D: mean Euclidean distance of each point to its
    three nearest valid neighbours (itself excluded), by brute force."""
    p = np.asarray(points, dtype=np.float64)
    n = p.shape[0]
    valid = np.ones(n, dtype=bool) if valid is None else np.asarray(valid, dtype=bool)
    out = np.full(n, INVALID_SCALE)
    cand = p[valid]
    cidx = np.nonzero(valid)[0]
    for s in range(0, n, 512):
        q = p[s:s + 512]
        d2 = ((q[:, None, :] - cand[None, :, :]) ** 2).sum(axis=2)
        self_hit = cidx[None, :] == np.arange(s, s + q.shape[0])[:, None]
        d2[self_hit] = np.inf
        k = min(3, d2.shape[1])
        if k == 0:
            continue
        near = np.sort(d2, axis=1)[:, :k]
        fin = np.isfinite(near)
        cnt = fin.sum(axis=1)
        dist = np.where(fin, np.sqrt(np.where(fin, near, 0.0)), 0.0).sum(axis=1)
        out[s:s + q.shape[0]] = np.where(cnt > 0, dist / np.maximum(cnt, 1), INVALID_SCALE)
    return out


def unproject(depth, image, cam, stride, opacity=0.5):
    """The unprojection of Sec. III-D.  Raw Gaussian parameters (means,
    log_scales, quats, logit_opacities,
    sh [n, 1, 3]) of the unprojected grid.  depth [h, w], image [3, h, w]
    over the camera's region of interest."""
    depth = np.asarray(depth, dtype=np.float64)
    image = np.asarray(image, dtype=np.float64)
    rx, ry, rw, rh = cam.roi if getattr(cam, "roi", None) is not None else (0, 0, cam.width, cam.height)
    nx, ny = grid_shape(rw, rh, stride)
    ys, xs = np.meshgrid(np.arange(ny) * stride, np.arange(nx) * stride, indexing="ij")
    xs, ys = xs.ravel(), ys.ravel()
    d = depth[ys, xs]
    ok = np.isfinite(d) & (d > 0)
    z = np.where(ok, d, 1.0)
    X = (xs + rx + 0.5 - float(cam.cx)) / float(cam.fx) * z
    Y = (ys + ry + 0.5 - float(cam.cy)) / float(cam.fy) * z
    means = np.stack([X, Y, z], axis=1)
    scale = knn3_mean_distance(means, ok)
    n = means.shape[0]
    quats = np.zeros((n, 4))
    quats[:, 0] = 1.0
    logit = np.where(ok, np.log(opacity / (1.0 - opacity)), INVALID_LOGIT)
    col = image[:, ys, xs].T
    sh = ((col - 0.5) / Y0)[:, None, :]
    return {"means": means, "log_scales": np.repeat(np.log(scale)[:, None], 3, axis=1),
            "quats": quats, "logit_opacities": logit, "sh": sh, "valid": ok}
