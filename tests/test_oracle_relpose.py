"""Pins of the relative-pose initialisation oracle (oracle/relpose.py):
nearest neighbours against scipy's k-d tree, unprojected points against
their own projection (closed form), colours through the C oracle's SH basis,
and the handling of invalid depths."""
import numpy as np
from scipy.spatial import cKDTree

import oracle
from oracle import relpose as RP


class _Cam:
    def __init__(self, W, H, fx, fy, cx, cy, roi=None):
        self.width, self.height, self.fx, self.fy, self.cx, self.cy = W, H, fx, fy, cx, cy
        self.roi = roi
        self.bg = (0.0, 0.0, 0.0)


def test_knn_matches_kdtree():
    rng = np.random.default_rng(1)
    p = rng.uniform(-1, 1, (700, 3))
    d, _ = cKDTree(p).query(p, k=4)          # column 0 is the point itself
    assert np.max(np.abs(RP.knn3_mean_distance(p) - d[:, 1:].mean(axis=1))) < 1e-14


def test_knn_ignores_invalid_points_and_handles_few():
    rng = np.random.default_rng(2)
    p = rng.uniform(-1, 1, (300, 3))
    valid = rng.random(300) < 0.7
    got = RP.knn3_mean_distance(p, valid)
    tree = cKDTree(p[valid])
    d, i = tree.query(p, k=4)
    vidx = np.nonzero(valid)[0]
    for k in range(300):
        nb = [dd for dd, ii in zip(d[k], i[k]) if vidx[ii] != k][:3]
        assert abs(got[k] - np.mean(nb)) < 1e-14
    two = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0], [9.0, 9.0, 9.0]])
    got = RP.knn3_mean_distance(two, np.array([True, True, False]))
    assert np.allclose(got[:2], 5.0)          # one valid neighbour each
    # an invalid point still gets the mean over the (two) valid points
    assert abs(got[2] - (np.linalg.norm(two[2] - two[0]) + np.linalg.norm(two[2] - two[1])) / 2) < 1e-12
    one = RP.knn3_mean_distance(two[:1])
    assert one[0] == RP.INVALID_SCALE


def test_unprojected_points_project_to_their_pixel_centres():
    rng = np.random.default_rng(3)
    cam = _Cam(64, 48, 55.0, 57.0, 31.7, 24.2, roi=(16, 16, 40, 30))
    depth = rng.uniform(1.0, 5.0, (30, 40))
    image = rng.uniform(0, 1, (3, 30, 40))
    out = RP.unproject(depth, image, cam, 3, opacity=0.1)
    nx, ny = RP.grid_shape(40, 30, 3)
    assert out["means"].shape == (nx * ny, 3)
    m = out["means"]
    u = cam.fx * m[:, 0] / m[:, 2] + cam.cx - 0.5
    v = cam.fy * m[:, 1] / m[:, 2] + cam.cy - 0.5
    ys, xs = np.meshgrid(np.arange(ny) * 3, np.arange(nx) * 3, indexing="ij")
    assert np.max(np.abs(u - (xs.ravel() + 16))) < 1e-12
    assert np.max(np.abs(v - (ys.ravel() + 16))) < 1e-12
    assert np.array_equal(m[:, 2], depth[ys.ravel(), xs.ravel()])
    # colour through the SH basis of degree 0 (the C oracle's) gives the pixel back
    y0 = oracle.sh_basis(0, np.array([0.0, 0.0, 1.0]))[0]
    col = out["sh"][:, 0, :] * y0 + 0.5
    assert np.max(np.abs(col - image[:, ys.ravel(), xs.ravel()].T)) < 1e-14
    assert np.allclose(out["logit_opacities"], np.log(0.1 / 0.9))
    assert np.array_equal(out["quats"], np.tile([1.0, 0, 0, 0], (nx * ny, 1)))
    assert np.allclose(np.exp(out["log_scales"][:, 0]), RP.knn3_mean_distance(m))


def test_invalid_depths():
    cam = _Cam(8, 8, 8.0, 8.0, 4.0, 4.0)
    depth = np.full((8, 8), 2.0)
    depth[0, 0] = 0.0
    depth[0, 2] = np.nan
    out = RP.unproject(depth, np.full((3, 8, 8), 0.5), cam, 2)
    assert not out["valid"][0] and not out["valid"][1] and out["valid"][2:].all()
    assert out["logit_opacities"][0] == RP.INVALID_LOGIT and out["means"][0, 2] == 1.0
    assert np.exp(out["log_scales"][0, 0]) > 0
