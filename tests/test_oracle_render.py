"""Pins of the oracle's forward pass: closed forms of projected Gaussians
(Sec. III-A, Eq. (1)-(4)), invariants of the compositing, brute force
against the tiled path, and symmetries of the whole render."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_2410_08743_amd import synthetic as S

C0 = 1.0 / (2.0 * np.sqrt(np.pi))
EPS = 0.3          # dilation added to the 2D covariance
TILE = 16


def _scene(means, scales, quats, opac, colors, degree=0):
    n = len(means)
    sh = np.zeros((n, (degree + 1) ** 2, 3))
    sh[:, 0, :] = (np.asarray(colors) - 0.5) / C0
    return S.GaussianSet(np.asarray(means, float), np.asarray(scales, float),
                         np.asarray(quats, float), np.asarray(opac, float), sh, degree)


def _identity():
    return np.concatenate([np.eye(3), np.zeros((3, 1))], 1)


def _radius(cov):
    a, b, c = cov
    mid = 0.5 * (a + c)
    lam = mid + np.sqrt(max(0.1, mid * mid - (a * c - b * b)))
    return int(np.ceil(3 * np.sqrt(lam)))


def _rect_mask(u, v, r, W, H):
    gw, gh = (W + 15) // 16, (H + 15) // 16
    x0 = min(max(int(np.floor((u - r) / 16)), 0), gw)
    x1 = min(max(int(np.floor((u + r + 15) / 16)), 0), gw)
    y0 = min(max(int(np.floor((v - r) / 16)), 0), gh)
    y1 = min(max(int(np.floor((v + r + 15) / 16)), 0), gh)
    m = np.zeros((H, W), bool)
    m[y0 * 16:y1 * 16, x0 * 16:x1 * 16] = True
    return m


def _alpha_map(u, v, conic, o, W, H):
    jj, ii = np.mgrid[0:H, 0:W].astype(float)
    dx, dy = u - ii, v - jj
    A, B, Cc = conic
    power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
    alpha = np.minimum(0.99, o * np.exp(power))
    alpha[(power > 0) | (alpha < 1.0 / 255.0)] = 0.0
    return alpha


def test_single_isotropic_gaussian_closed_form():
    # sigma^2 = (f s / z)^2 + 0.3 = 100; the tile rect (3 sigma) cuts pixels
    # whose alpha would still exceed 1/255 (up to 3.33 sigma at o = 0.99).
    W = H = 128
    f, z = 128.0, 4.0
    s = np.sqrt(100.0 - EPS) * z / f
    col, o, bg = [0.9, 0.4, 0.2], 0.99, (0.1, 0.2, 0.3)
    cam = S.Camera(W, H, f, f, 64.0, 64.0, bg=bg)
    sc = _scene([[0, 0, 0]], [[s, s, s]], [[1, 0, 0, 0]], [o], [col])
    pose = _identity()
    pose[2, 3] = z
    out = oracle.render(sc, cam, pose)
    u = v = 63.5
    sig2 = (f * s / z) ** 2 + EPS
    r = int(np.ceil(3 * np.sqrt(sig2 + np.sqrt(0.1))))
    mask = _rect_mask(u, v, r, W, H)
    jj, ii = np.mgrid[0:H, 0:W].astype(float)
    alpha = o * np.exp(-((u - ii) ** 2 + (v - jj) ** 2) / (2 * sig2))
    alpha = np.where(mask & (alpha >= 1 / 255), np.minimum(alpha, 0.99), 0.0)
    for ch in range(3):
        ref = col[ch] * alpha + (1 - alpha) * bg[ch]
        assert np.max(np.abs(out["image"][ch] - ref)) < 1e-12
    assert np.max(np.abs(out["T_final"] - (1 - alpha))) < 1e-12
    # the rect really does cut visible alpha here
    outside = (~mask) & (o * np.exp(-((u - ii) ** 2 + (v - jj) ** 2) / (2 * sig2)) >= 1 / 255)
    assert outside.any()


def test_anisotropic_rotated_gaussian_closed_form():
    W, H = 96, 80
    f, z = 100.0, 5.0
    th = 0.6
    R = Rotation.from_rotvec([0, 0, th]).as_matrix()
    sxyz = np.array([0.3, 0.08, 0.05])
    q = [np.cos(th / 2), 0, 0, np.sin(th / 2)]
    cam = S.Camera(W, H, f, f, 48.0, 40.0)
    sc = _scene([[0, 0, 0]], [sxyz], [q], [0.7], [[0.5, 0.6, 0.7]])
    pose = _identity()
    pose[2, 3] = z
    sp = oracle.preprocess(sc, cam, pose)[0]
    Sig = R @ np.diag(sxyz ** 2) @ R.T
    cov = (f / z) ** 2 * Sig[:2, :2] + EPS * np.eye(2)
    assert np.allclose(sp["cov"], [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=0, atol=1e-12)
    conic = np.linalg.inv(cov)
    assert np.allclose(sp["conic"], [conic[0, 0], conic[0, 1], conic[1, 1]], rtol=0, atol=1e-13)
    out = oracle.render(sc, cam, pose)
    u, v = 47.5, 39.5
    alpha = _alpha_map(u, v, (conic[0, 0], conic[0, 1], conic[1, 1]), 0.7, W, H)
    alpha *= _rect_mask(u, v, _radius(sp["cov"]), W, H)
    assert np.max(np.abs(out["image"][0] - 0.5 * alpha)) < 1e-12
    assert np.max(np.abs(out["T_final"] - (1 - alpha))) < 1e-12


def test_off_axis_isotropic_covariance_closed_form():
    rng = np.random.default_rng(21)
    W, H, f = 200, 150, 180.0
    cam = S.Camera(W, H, f, f, 100.0, 75.0)
    n = 200
    z = rng.uniform(1, 6, n)
    x = rng.uniform(-0.5, 0.5, n) * z
    y = rng.uniform(-0.4, 0.4, n) * z
    s = rng.uniform(0.01, 0.2, n)
    sc = _scene(np.stack([x, y, z], 1), np.stack([s, s, s], 1), S.random_quats(rng, n),
                np.full(n, 0.5), np.full((n, 3), 0.5))
    sp = oracle.preprocess(sc, cam, _identity())
    a = s ** 2 * (f / z) ** 2 * (1 + x * x / z ** 2) + EPS
    b = s ** 2 * (f / z) ** 2 * (x * y / z ** 2)
    c = s ** 2 * (f / z) ** 2 * (1 + y * y / z ** 2) + EPS
    assert np.allclose(sp["cov"][:, 0], a, rtol=1e-12)
    assert np.allclose(sp["cov"][:, 1], b, rtol=1e-10, atol=1e-14)
    assert np.allclose(sp["cov"][:, 2], c, rtol=1e-12)
    assert np.allclose(sp["u"], f * x / z + 100.0 - 0.5, rtol=0, atol=1e-12)
    assert np.allclose(sp["v"], f * y / z + 75.0 - 0.5, rtol=0, atol=1e-12)
    assert np.array_equal(sp["depth_key"], z.astype(np.float32))


def test_two_gaussians_composite_closed_form():
    W = H = 64
    f = 64.0
    cam = S.Camera(W, H, f, f, 32.0, 32.0, bg=(0.25, 0.5, 0.75))
    s1, s2 = 0.08, 0.2
    c1, c2 = [1.0, 0.0, 0.2], [0.1, 0.9, 0.3]
    o1, o2 = 0.6, 0.85
    sc = _scene([[0.05, 0, 0], [-0.1, 0.05, 2]], [[s1] * 3, [s2] * 3], [[1, 0, 0, 0]] * 2,
                [o1, o2], [c1, c2])
    pose = _identity()
    pose[2, 3] = 3.0
    out = oracle.render(sc, cam, pose)
    sp = oracle.preprocess(sc, cam, pose)
    alphas = []
    for k in range(2):
        s = sp[k]
        al = _alpha_map(s["u"], s["v"], s["conic"], s["opacity"], W, H)
        al *= _rect_mask(s["u"], s["v"], _radius(s["cov"]), W, H)
        alphas.append(al)
    a1, a2 = alphas
    for ch in range(3):
        ref = c1[ch] * a1 + c2[ch] * a2 * (1 - a1) + cam.bg[ch] * (1 - a1) * (1 - a2)
        assert np.max(np.abs(out["image"][ch] - ref)) < 1e-12


def test_transmittance_cutoff_stack():
    # Five Gaussians with alpha = 0.8 at the centre pixel leave T = 0.2^5 =
    # 3.2e-4; the sixth would take it to 6.4e-5 < 1e-4, so compositing stops
    # before it and n_contrib = 5.
    W = H = 32
    f = 32.0
    cam = S.Camera(W, H, f, f, 16.5, 16.5, bg=(0.3, 0.3, 0.3))   # pixel (16, 16) on the axis
    cols = np.array([[0.1 * k, 1 - 0.1 * k, 0.5] for k in range(7)])
    zs = 2.0 + 0.5 * np.arange(7)
    sc = _scene(np.stack([np.zeros(7), np.zeros(7), zs - 4.0], 1), np.full((7, 3), 0.05),
                [[1, 0, 0, 0]] * 7, np.full(7, 0.8), cols)
    pose = _identity()
    pose[2, 3] = 4.0
    out = oracle.render(sc, cam, pose)
    assert out["n_contrib"][16, 16] == 5
    ref = sum(cols[k] * 0.8 * 0.2 ** k for k in range(5)) + 0.2 ** 5 * 0.3
    assert np.max(np.abs(out["image"][:, 16, 16] - ref)) < 1e-12
    assert abs(out["T_final"][16, 16] - 0.2 ** 5) < 1e-15
    tr = oracle.pixel_trace(sc, cam, pose, 16, 16)
    assert list(tr["blended"]) == [1, 1, 1, 1, 1, 0]


def test_empty_scene_renders_background():
    cam = S.Camera(40, 24, 30.0, 30.0, 20.0, 12.0, bg=(0.2, 0.4, 0.6))
    sc = _scene(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 4)), np.zeros(0), np.zeros((0, 3)))
    out = oracle.render(sc, cam, _identity())
    for ch in range(3):
        assert np.all(out["image"][ch] == cam.bg[ch])
    assert np.all(out["T_final"] == 1.0) and np.all(out["n_contrib"] == 0)


def _small(seed, degree, W=70, H=52, n=60, roi=None):
    cam = S.Camera(W, H, 60.0, 62.0, W / 2 + 0.3, H / 2 - 0.7, roi=roi, bg=(0.1, 0.05, 0.2))
    sc = S.random_scene(seed, n, degree, cam, depth=(0.1, 5.0))
    # float64 rotation, orthonormal to rounding, so that R^-1 = R^T holds
    pose = S.perturb_pose(S.identity_pose(), 2.0, 0.05, S.rng_for(seed, 7))
    return sc, cam, pose


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
@pytest.mark.parametrize("seed", [1, 2])
def test_brute_force_equals_tiled(degree, seed):
    sc, cam, pose = _small(seed + 10 * degree, degree)
    a = oracle.render(sc, cam, pose)
    b = oracle.render_brute(sc, cam, pose)
    assert np.array_equal(a["image"], b["image"])
    assert np.array_equal(a["T_final"], b["T_final"])


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_compositing_invariants(seed):
    sc, cam, pose = _small(seed, 3, n=120)
    out = oracle.render(sc, cam, pose)
    assert np.all(out["T_final"] >= 1e-4) and np.all(out["T_final"] <= 1.0)
    rng = np.random.default_rng(seed)
    for _ in range(40):
        px, py = int(rng.integers(0, cam.width)), int(rng.integers(0, cam.height))
        tr = oracle.pixel_trace(sc, cam, pose, px, py)
        bl = tr[tr["blended"] == 1]
        # blended alphas within [1/255, 0.99]; skipped ones below 1/255 or the stop
        assert np.all(bl["alpha"] >= 1 / 255) and np.all(bl["alpha"] <= 0.99)
        # transmittance is the running product and never increases
        T = np.concatenate([bl["T_before"], [out["T_final"][py, px]]])
        assert np.all(np.diff(T) <= 0)
        assert np.allclose(T[1:], np.cumprod(1 - bl["alpha"]), rtol=1e-13, atol=0)
        # weights plus the final transmittance sum to one
        assert abs(np.sum(bl["alpha"] * bl["T_before"]) + out["T_final"][py, px] - 1) < 1e-12
        skipped = tr[tr["blended"] == 0]
        if len(skipped):
            last = tr[-1]
            for e in skipped[:-1] if last["blended"] == 0 else skipped:
                assert e["alpha"] < 1 / 255 or e["power"] > 0 or \
                    e["T_before"] * (1 - e["alpha"]) < 1e-4
        nb = int(out["n_contrib"][py, px])
        assert nb == (int(bl["position"][-1]) + 1 if len(bl) else 0)
        # a stop can only be the last evaluated entry
        stops = [i for i, e in enumerate(tr) if e["blended"] == 0 and e["alpha"] >= 1 / 255
                 and e["power"] <= 0]
        assert all(i == len(tr) - 1 for i in stops)


def test_roi_crop_equals_full_image_crop():
    sc, cam, pose = _small(31, 3, W=100, H=75, n=150)
    full = oracle.render(sc, cam, pose)
    for roi in [(16, 16, 48, 32), (32, 0, 68, 75), (0, 48, 37, 27), (80, 64, 20, 11)]:
        crop = oracle.render(sc, cam.with_roi(roi), pose)
        x, y, w, h = roi
        assert np.array_equal(crop["image"], full["image"][:, y:y + h, x:x + w])
        assert np.array_equal(crop["n_contrib"], full["n_contrib"][y:y + h, x:x + w])


def test_input_permutation_leaves_image_unchanged():
    sc, cam, pose = _small(41, 2, n=90)
    perm = np.random.default_rng(41).permutation(sc.n)
    a = oracle.render(sc, cam, pose)
    b = oracle.render(sc.subset(perm), cam, pose)
    sp = oracle.preprocess(sc, cam, pose)
    assert len(np.unique(sp["depth_key"])) == sc.n
    assert np.array_equal(a["image"], b["image"])


@pytest.mark.parametrize("degree", [0, 3])
def test_translation_gauge(degree):
    # moving every Gaussian by v and the camera with it leaves the image unchanged
    sc, cam, pose = _small(51, degree, n=80)
    v = np.array([0.3, -0.2, 0.7])
    moved = S.GaussianSet(sc.means.astype(float) + v, sc.scales, sc.quats, sc.opacities, sc.sh,
                          degree)
    pose2 = pose.copy()
    pose2[:, 3] = pose[:, 3] - pose[:, :3] @ v
    a = oracle.render(sc, cam, pose)
    b = oracle.render(moved, cam, pose2)
    assert np.max(np.abs(a["image"] - b["image"])) < 1e-11


def test_rigid_rotation_invariance_sh0():
    # rotating the world (means and orientations) and the camera together
    # leaves a view-independent image unchanged: pins R_c and R(q) in Eq. (2)
    sc, cam, pose = _small(61, 0, n=80)
    Q = Rotation.from_rotvec([0.4, -0.3, 0.9])
    means = Q.apply(sc.means.astype(float))
    qs = sc.quats.astype(float)
    rq = (Q * Rotation.from_quat(np.stack([qs[:, 1], qs[:, 2], qs[:, 3], qs[:, 0]], 1))).as_quat()
    quats = np.stack([rq[:, 3], rq[:, 0], rq[:, 1], rq[:, 2]], 1)
    rot = S.GaussianSet(means, sc.scales, quats, sc.opacities, sc.sh, 0)
    pose2 = pose.copy()
    pose2[:, :3] = pose[:, :3] @ Q.as_matrix().T
    a = oracle.render(sc, cam, pose)
    b = oracle.render(rot, cam, pose2)
    assert np.max(np.abs(a["image"] - b["image"])) < 1e-9


def _brute_instances(splats, gw, gh, base=0, voff=0):
    pairs = []
    for i, s in enumerate(splats):
        if not s["rendered"]:
            continue
        x0, y0, x1, y1 = s["rect"]
        d = int(np.array(s["depth_key"], dtype=np.float32).view(np.uint32))
        for ty in range(gh):
            for tx in range(gw):
                if x0 <= tx < x1 and y0 <= ty < y1:
                    pairs.append((((base + ty * gw + tx) << 32) | d, voff + i))
    return pairs


def test_bin_sort_matches_brute_force_two_views():
    sc, cam, pose = _small(71, 1, n=70)
    cam2 = cam.with_roi((16, 16, 40, 30))
    pose2 = S.random_pose_near_identity(72, 3.0, 0.1).astype(np.float64)
    s1 = oracle.preprocess(sc, cam, pose)
    s2 = oracle.preprocess(sc, cam2, pose2)
    t1, t2 = oracle.tiles_of(cam), oracle.tiles_of(cam2)
    keys, vals = oracle.bin_sort([s1, s2], [t1, t2])
    pairs = _brute_instances(s1, *t1) + _brute_instances(s2, *t2, base=t1[0] * t1[1], voff=sc.n)
    pairs.sort()
    assert len(keys) == len(pairs) == oracle.count_instances([s1, s2])
    assert np.array_equal(keys, np.array([p[0] for p in pairs], dtype=np.uint64))
    assert np.array_equal(vals, np.array([p[1] for p in pairs], dtype=np.uint32))
    ntiles = t1[0] * t1[1] + t2[0] * t2[1]
    rng_ = oracle.tile_ranges(keys, ntiles)
    tiles = keys >> np.uint64(32)
    for t in range(ntiles):
        st, en = rng_[t]
        idx = np.nonzero(tiles == t)[0]
        if len(idx) == 0:
            assert st == en == 0
        else:
            assert st == idx[0] and en == idx[-1] + 1 and en - st == len(idx)
