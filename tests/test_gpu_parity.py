"""HIP path vs the FP64 oracle, stage by stage, through the C ABI.

Bars: per-Gaussian records to rounding; sort keys, values and tile ranges bit
for bit; images within 1e-4 absolute on every pixel the oracle does not flag
as straddling an FP32/FP64 decision (straddling pixels are counted and must
be rare); gradients within 1e-3 relative L2 per parameter group and per pose
block (rho, phi), and element by element within 1e-3 of the group's largest
oracle value.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_08743_amd import render as R
from paper_2410_08743_amd import synthetic as S
from tests.parity_util import (assert_grad_close, assert_sorted_match, f32_camera,
                                 max_rel_inf, random_case, rel_l2, unpack_rect)

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _case(name):
    if name == "tiny":
        wl = S.tiny()
        return wl.scene, f32_camera(wl.camera), wl.pose
    if name == "sh0":
        return random_case(11, 0, 96, 64, 300)
    if name == "sh1-ragged":
        return random_case(12, 1, 70, 53, 250)
    if name == "sh2-near":
        return random_case(13, 2, 80, 80, 300, depth=(0.05, 4.0), lateral=2.0)
    if name == "sh3-roi":
        return random_case(14, 3, 120, 90, 400, roi=(32, 16, 61, 50))
    if name == "sh3-dense":
        return random_case(15, 3, 128, 96, 3000, depth=(1.0, 8.0))
    if name == "sh1-thin":
        # needle-like splats (one axis x0.02, one x3) and opacities down to
        # just above 1/255: the per-entry culling bound at its margins
        sc, cam, pose = random_case(16, 1, 96, 80, 600, depth=(0.5, 5.0))
        rng = S.rng_for(16, 9)
        k = rng.integers(0, 3, sc.n)
        idx = np.arange(sc.n)
        sc.scales[idx, k] *= np.float32(0.02)
        sc.scales[idx, (k + 1) % 3] *= np.float32(3.0)
        sc.opacities[:] = rng.uniform(0.005, 0.99, sc.n).astype(np.float32)
        return sc, cam, pose
    if name == "sh1-opaque":
        # opacities of 0.95-0.999: alpha reaches the 0.99 clamp near the
        # splats' centres, and most batches take the rasterizers' clamping
        # walk rather than the walk for splats that cannot reach it
        sc, cam, pose = random_case(18, 1, 96, 72, 500, depth=(0.8, 5.0))
        rng = S.rng_for(18, 9)
        sc.opacities[:] = rng.uniform(0.95, 0.999, sc.n).astype(np.float32)
        return sc, cam, pose
    if name == "sh2-deep":
        # tile lists of 1000-1200 entries, pixels compositing past several
        # cuts: the backward's chunks start from the forward's cut states
        return random_case(17, 2, 64, 48, 9000, depth=(1.0, 8.0))
    if name == "sh2-deeper":
        # lists of ~2500 entries: more than kMaxChunks chunks' worth, so the
        # last chunk of every tile is longer than the others
        return random_case(17, 2, 64, 48, 20000, depth=(1.0, 8.0))
    raise KeyError(name)


CASES = ["tiny", "sh0", "sh1-ragged", "sh2-near", "sh3-roi", "sh3-dense", "sh1-thin", "sh1-opaque",
         "sh2-deep", "sh2-deeper"]
# chunk length of the backward's work items and their most per tile
CHUNK = 128
MAX_CHUNKS = 16


def _gpu(sc, cams, poses, up=None, cap=0, want=("means", "scales", "quats", "opacities", "sh")):
    g = R.GaussianParams.from_set(sc, DEV)
    P = torch.tensor(np.stack(poses), device=DEV, dtype=torch.float32)
    rast = R.Rasterizer(0, capacity=cap)
    img, alpha = rast.forward(g, cams, P, alphas=True)
    out = {"images": [t.cpu().numpy() for t in R.split_images(img, cams)],
           "alpha": alpha.cpu().numpy(), "rast": rast, "g": g, "P": P}
    if up is not None:
        dl = torch.tensor(np.concatenate([u.ravel() for u in up]), device=DEV)
        gr = rast.backward(g, cams, P, dl, want=want)
        out.update({k: v.cpu().numpy() for k, v in gr.items()})
    torch.cuda.synchronize()
    return out


def _tiles(cam):
    gw, gh = oracle.tiles_of(cam)
    return range(gw * gh)


def _upstream(seed, cam):
    x, y, w, h = cam.region()
    return S.upstream(seed, (3, h, w))


@pytest.mark.parametrize("name", CASES)
def test_preprocess_records(name):
    sc, cam, pose = _case(name)
    run = _gpu(sc, [cam], [pose])
    rast, g = run["rast"], run["g"]
    ref = oracle.preprocess(sc, cam, pose)
    geom = rast.inspect(g, [cam], "geom").cpu().numpy().reshape(-1, 8)
    col = rast.inspect(g, [cam], "color").cpu().numpy().reshape(-1, 4)
    rect = unpack_rect(rast.inspect(g, [cam], "rect", torch.int32).cpu().numpy())
    depth = rast.inspect(g, [cam], "depth", torch.int32).cpu().numpy().view(np.uint32)
    tiles = rast.inspect(g, [cam], "tiles", torch.int32).cpu().numpy()
    solid = (ref["fragile"] == 0)
    ren = (ref["rendered"] == 1) & solid
    print(f"{name}: n={sc.n} rendered={int(ren.sum())} fragile={int((~solid).sum())}")
    assert np.array_equal(depth, ref["depth_key"].view(np.uint32))
    ref_tiles = np.where(ref["rendered"] == 1,
                         (ref["rect"][:, 2] - ref["rect"][:, 0]) * (ref["rect"][:, 3] - ref["rect"][:, 1]), 0)
    assert np.array_equal(tiles[solid], ref_tiles[solid])
    assert np.array_equal(rect[ren], ref["rect"][ren])
    u = geom[:, 0].astype(np.float64) + geom[:, 2]
    v = geom[:, 1].astype(np.float64) + geom[:, 3]
    assert np.max(np.abs(u[ren] - ref["u"][ren])) < 1e-9 * max(1.0, np.abs(ref["u"][ren]).max())
    assert np.max(np.abs(v[ren] - ref["v"][ren])) < 1e-9 * max(1.0, np.abs(ref["v"][ren]).max())
    # stored in base 2 with the -1/2 folded in: (A2, B2, C2) = -log2(e) (A/2, B, C/2)
    log2e = 1.0 / np.log(2.0)
    conic = geom[:, 4:7].astype(np.float64) * np.array([-2.0, -1.0, -2.0]) / log2e
    assert np.max(np.abs(conic[ren] - ref["conic"][ren]) / np.abs(ref["conic"][ren]).max(1, keepdims=True)) < 1e-6
    o = np.exp2(geom[:, 7].astype(np.float64))
    assert np.max(np.abs(o[ren] - sc.opacities[ren]) / sc.opacities[ren]) < 1e-6
    assert np.max(np.abs(col[ren, :3] - ref["color"][ren])) < 2e-6


# capacities above 6M instances (6 << 20) take the 2048-key blocks of the
# instance emission and sort
@pytest.mark.parametrize("cap", [0, (6 << 20) + 1])
@pytest.mark.parametrize("name", CASES)
def test_keys_sort_and_ranges_bit_exact(name, cap):
    sc, cam, pose = _case(name)
    run = _gpu(sc, [cam], [pose], cap=cap)
    rast, g = run["rast"], run["g"]
    ref = oracle.preprocess(sc, cam, pose)
    gw, gh = oracle.tiles_of(cam)
    rkeys, rvals = oracle.bin_sort([ref], [(gw, gh)])
    M, ovf = rast.instances()
    assert not ovf
    keys, vals = _sorted_instances(rast, g, [cam], M)
    fragile = np.nonzero(ref["fragile"])[0].astype(np.uint32)
    assert_sorted_match(keys, vals, rkeys, rvals, fragile)
    if len(fragile) == 0:
        ranges = rast.inspect(g, [cam], "ranges", torch.int32).cpu().numpy().view(np.uint32)
        assert np.array_equal(ranges.reshape(-1, 2), oracle.tile_ranges(rkeys, gw * gh))


@pytest.mark.parametrize("cap", [0, (6 << 20) + 1])
def test_depth_ties_and_long_runs_bit_exact(cap):
    """Tile runs several times longer than the per-tile depth sort keeps in
    LDS (its chunked global-memory path), with depth ties everywhere: 25000
    Gaussians at three depths only, seen at the identity pose, so that the
    camera-frame z of each is its mean's z exactly and equal keys must come
    out in index order."""
    sc, cam, _ = random_case(18, 0, 48, 32, 25000, depth=(2.0, 5.0))
    z = np.array([2.0, 3.0, 4.5], np.float32)[S.rng_for(18, 5).integers(0, 3, sc.n)]
    sc.means[:, :2] *= (z / sc.means[:, 2])[:, None]
    sc.means[:, 2] = z
    pose = S.identity_pose()
    run = _gpu(sc, [cam], [pose], cap=cap)
    rast, g = run["rast"], run["g"]
    ref = oracle.preprocess(sc, cam, pose)
    gw, gh = oracle.tiles_of(cam)
    rkeys, rvals = oracle.bin_sort([ref], [(gw, gh)])
    M, ovf = rast.instances()
    assert not ovf
    keys, vals = _sorted_instances(rast, g, [cam], M)
    tile_len = np.bincount((rkeys >> np.uint64(32)).astype(np.int64), minlength=gw * gh)
    assert tile_len.max() > 2 * 2048
    assert len(np.unique(ref["depth_key"])) <= 3
    fragile = np.nonzero(ref["fragile"])[0].astype(np.uint32)
    assert_sorted_match(keys, vals, rkeys, rvals, fragile)


def test_keys_bit_exact_two_views():
    sc, cam0, pose0 = random_case(16, 2, 96, 64, 700)
    cam1 = f32_camera(S.Camera(80, 48, 75.0, 70.0, 40.5, 23.75, roi=(16, 16, 50, 32)))
    pose1 = S.random_pose_near_identity(17, 3.0, 0.1)
    run = _gpu(sc, [cam0, cam1], [pose0, pose1])
    rast, g = run["rast"], run["g"]
    s0, s1 = oracle.preprocess(sc, cam0, pose0), oracle.preprocess(sc, cam1, pose1)
    assert not s0["fragile"].any() and not s1["fragile"].any()
    rkeys, rvals = oracle.bin_sort([s0, s1], [oracle.tiles_of(cam0), oracle.tiles_of(cam1)])
    M, ovf = rast.instances()
    assert not ovf and M == len(rkeys)
    keys, vals = _sorted_instances(rast, g, [cam0, cam1], M)
    assert np.array_equal(keys, rkeys) and np.array_equal(vals, rvals)


def _sorted_instances(rast, g, cams, M):
    """The GPU's sorted instances as 64-bit (tile << 32 | depth bits) keys:
    the instance sort carries tile ids; the depth bits are the splat's."""
    tiles = rast.inspect(g, cams, "keys", torch.int32).cpu().numpy().view(np.uint32)[:M]
    vals = rast.inspect(g, cams, "values", torch.int32).cpu().numpy().view(np.uint32)[:M]
    depth = rast.inspect(g, cams, "depth", torch.int32).cpu().numpy().view(np.uint32)
    keys = (tiles.astype(np.uint64) << np.uint64(32)) | depth[vals].astype(np.uint64)
    return keys, vals


def _image_check(img, ref, name, max_straddle=2e-3):
    strad = ref["straddle"]
    err = np.abs(img - ref["image"]).max(axis=0)
    ok = ~strad
    worst = float(err[ok].max()) if ok.any() else 0.0
    print(f"{name}: max |image - oracle| = {worst:.2e}, straddling pixels {int(strad.sum())}/{strad.size}")
    assert strad.mean() <= max_straddle
    assert worst <= 1e-4


@pytest.mark.parametrize("name", CASES)
def test_image_parity(name):
    sc, cam, pose = _case(name)
    run = _gpu(sc, [cam], [pose])
    ref = oracle.render(sc, cam, pose)
    img = run["images"][0]
    _image_check(img, ref, name)
    ok = ~ref["straddle"]
    alpha = run["alpha"].reshape(ref["T_final"].shape)
    assert np.max(np.abs((1 - alpha)[ok] - ref["T_final"][ok])) <= 1e-5
    nc = run["rast"].inspect(run["g"], [cam], "ncontrib", torch.int32).cpu().numpy()
    nc = nc.reshape(ref["n_contrib"].shape)
    assert np.mean(nc[ok] == ref["n_contrib"][ok]) >= 0.999


@pytest.mark.parametrize("name", CASES)
def test_backward_parity(name):
    sc, cam, pose = _case(name)
    up = _upstream(21, cam)
    run = _gpu(sc, [cam], [pose], up=[up])
    ref = oracle.backward(sc, cam, pose, up)
    g2 = run["rast"].inspect(run["g"], [cam], "grad2d").cpu().numpy().reshape(-1, 9)
    pairs = {"splat2d": (g2, ref["splat2d"])}
    for k in ("means", "scales", "quats", "opacities", "sh"):
        pairs[k] = (run[k], ref[k])
    pairs["rho"] = (run["pose"][0, :3], ref["pose"][:3])
    pairs["phi"] = (run["pose"][0, 3:], ref["pose"][3:])
    print(name, {k: f"{rel_l2(a, b):.1e}/{max_rel_inf(a, b):.1e}" for k, (a, b) in pairs.items()})
    for k, (a, b) in pairs.items():
        assert_grad_close(a, b, k)


@pytest.mark.parametrize("name", ["sh2-deep", "sh2-deeper"])
def test_long_lists_are_cut(name):
    """The deep cases exercise what they are for: lists longer than a chunk
    (and, for the deeper one, than kMaxChunks chunks), with pixels that
    composite past a cut."""
    sc, cam, pose = _case(name)
    ref = oracle.preprocess(sc, cam, pose)
    gw, gh = oracle.tiles_of(cam)
    rkeys, _ = oracle.bin_sort([ref], [(gw, gh)])
    ln = np.diff(oracle.tile_ranges(rkeys, gw * gh), axis=1).ravel()
    assert (ln > CHUNK).all()
    if name == "sh2-deeper":
        assert (ln > MAX_CHUNKS * CHUNK).all()
    nc = oracle.render(sc, cam, pose)["n_contrib"]
    assert (nc > 4 * CHUNK).mean() > 0.2   # past four cuts


def test_multiview_batch_equals_single_views():
    sc, cam0, pose0 = random_case(31, 3, 96, 64, 800)
    cam1 = f32_camera(S.Camera(80, 48, 75.0, 70.0, 40.5, 23.75, roi=(16, 0, 50, 48)))
    cam2 = f32_camera(S.Camera(64, 64, 60.0, 60.0, 32.0, 32.0, bg=(0.5, 0.5, 0.5)))
    pose1 = S.random_pose_near_identity(32, 3.0, 0.1)
    pose2 = S.random_pose_near_identity(33, 5.0, 0.1)
    cams, poses = [cam0, cam1, cam2], [pose0, pose1, pose2]
    ups = [_upstream(40 + k, c) for k, c in enumerate(cams)]
    both = _gpu(sc, cams, poses, up=ups)
    sums = {k: 0 for k in ("means", "scales", "quats", "opacities", "sh")}
    for k in range(3):
        one = _gpu(sc, [cams[k]], [poses[k]], up=[ups[k]])
        assert np.array_equal(both["images"][k], one["images"][0])
        assert np.array_equal(both["pose"][k], one["pose"][0])
        for key in sums:
            sums[key] = sums[key] + one[key].astype(np.float64)
    for key in sums:
        assert_grad_close(both[key], sums[key], key, rel=1e-6, elem=1e-6)


def test_batched_views_with_and_without_long_lists():
    """One launch holding a view with millions of instances (lists of
    thousands of entries, cut into chunks) and a small one gives each view
    the image and pose gradient it gets alone, bit for bit."""
    wl = S.joint()
    big = wl.camera
    small = S.Camera(1008, 756, 815.0, 815.0, 504.0, 378.0, roi=(400, 304, 160, 128))
    cams = [big, small]
    poses = [wl.extra["noisy_poses"][0], wl.extra["noisy_poses"][3]]
    g = R.GaussianParams.from_set(wl.scene, DEV)
    ups = [_upstream(60 + k, c) for k, c in enumerate(cams)]

    def run(cs, ps, us):
        P = torch.tensor(np.stack(ps), device=DEV, dtype=torch.float32)
        rast = R.Rasterizer(0)
        img, _ = rast.forward(g, cs, P)
        M, ovf = rast.instances()
        assert not ovf
        dl = torch.tensor(np.concatenate([u.ravel() for u in us]), device=DEV)
        gr = rast.backward(g, cs, P, dl, want=(), pose=True)
        torch.cuda.synchronize()
        return [t.cpu().numpy() for t in R.split_images(img, cs)], gr["pose"].cpu().numpy(), M

    imgs, pose, _ = run(cams, poses, ups)
    Ms = []
    for k in range(2):
        i1, p1, M1 = run([cams[k]], [poses[k]], [ups[k]])
        Ms.append(M1)
        assert np.array_equal(imgs[k], i1[0])
        assert np.array_equal(pose[k], p1[0])
    assert Ms[0] > 1000 * len(_tiles(big)) and Ms[1] < Ms[0] // 10


def test_pose_gradient_without_opacity_sum_is_bit_identical():
    """A backward that wants no opacity gradient reduces eight sums per
    entry instead of nine; every other 2D gradient component, and the pose
    gradient, come out bit for bit as with the opacity gradient."""
    sc, cam, pose = random_case(47, 3, 112, 80, 1500)
    up = _upstream(47, cam)
    outs = []
    for want in [(), ("opacities",)]:
        g = R.GaussianParams.from_set(sc, DEV)
        P = torch.tensor(pose[None], device=DEV, dtype=torch.float32)
        rast = R.Rasterizer(0)
        rast.forward(g, [cam], P)
        gr = rast.backward(g, [cam], P, torch.tensor(up.ravel(), device=DEV), want=want, pose=True)
        g2 = rast.inspect(g, [cam], "grad2d").cpu().numpy().reshape(-1, 9)
        torch.cuda.synchronize()
        outs.append((gr["pose"].cpu().numpy(), g2))
    (p0, a0), (p1, a1) = outs
    assert np.array_equal(p0, p1)
    keep = [0, 1, 2, 3, 4, 6, 7, 8]
    assert np.array_equal(a0[:, keep], a1[:, keep])
    assert np.all(a0[:, 5] == 0) and np.any(a1[:, 5] != 0)


def test_roi_equals_full_image_crop():
    sc, cam, pose = random_case(41, 3, 112, 80, 600)
    full = _gpu(sc, [cam], [pose])["images"][0]
    for roi in [(16, 16, 64, 48), (48, 0, 64, 80), (0, 32, 37, 21)]:
        crop = _gpu(sc, [cam.with_roi(roi)], [pose])["images"][0]
        x, y, w, h = roi
        assert np.array_equal(crop, full[:, y:y + h, x:x + w])


def test_bitwise_reproducible():
    sc, cam, pose = random_case(51, 3, 128, 96, 2000)
    up = _upstream(52, cam)
    a = _gpu(sc, [cam], [pose], up=[up])
    b = _gpu(sc, [cam], [pose], up=[up])
    assert np.array_equal(a["images"][0], b["images"][0])
    for k in ("means", "scales", "quats", "opacities", "sh", "pose"):
        assert np.array_equal(a[k], b[k]), k


def test_capacity_overflow_regrows_and_matches():
    sc, cam, pose = random_case(61, 2, 96, 64, 500)
    ref = _gpu(sc, [cam], [pose], cap=10_000_000)
    g = R.GaussianParams.from_set(sc, DEV)
    P = torch.tensor(pose[None], device=DEV)
    rast = R.Rasterizer(0, capacity=64)
    rast.forward(g, [cam], P, check=False)
    m, ovf = rast.instances()
    assert ovf and m > 64
    img, _ = rast.forward(g, [cam], P, check=True)
    assert rast.capacity >= m
    assert np.array_equal(R.split_images(img, [cam])[0].cpu().numpy(), ref["images"][0])


def test_empty_and_invisible_scenes_render_background():
    cam = f32_camera(S.Camera(48, 40, 40.0, 40.0, 24.0, 20.0, bg=(0.25, 0.5, 0.75)))
    empty = S.GaussianSet(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32),
                          np.zeros((0, 4), np.float32), np.zeros(0, np.float32),
                          np.zeros((0, 1, 3), np.float32), 0)
    behind, _, _ = random_case(71, 0, 48, 40, 50)
    behind.means[:, 2] = -np.abs(behind.means[:, 2]) - 1.0
    for sc in (empty, behind):
        up = _upstream(72, cam)
        run = _gpu(sc, [cam], [S.identity_pose()], up=[up])
        for ch in range(3):
            assert np.all(run["images"][0][ch] == np.float32(cam.bg[ch]))
        assert np.all(run["pose"] == 0)
        if sc.n:
            assert np.all(run["means"] == 0)


def test_l1_loss_kernel_per_view():
    # two views of different, non-tile-multiple sizes in one launch: each view
    # is normalised by its own value count
    rng = np.random.default_rng(81)
    cams = [S.Camera(101, 37, 90.0, 90.0, 50.0, 18.0), S.Camera(64, 48, 60.0, 60.0, 32.0, 24.0)]
    preds, targets = [], []
    for c in cams:
        a = rng.standard_normal(3 * c.width * c.height).astype(np.float32)
        b = a.copy()
        b[::5] = rng.standard_normal(len(b[::5])).astype(np.float32)
        preds.append(a)
        targets.append(b)
    loss, grads = R.loss_l1(cams, [torch.tensor(a, device=DEV) for a in preds],
                            [torch.tensor(b, device=DEV) for b in targets])
    loss = loss.cpu().numpy()
    for v in range(len(cams)):
        rv, rg = oracle.l1(preds[v], targets[v])
        g = grads[v].cpu().numpy()
        assert abs(float(loss[v]) - rv) <= 1e-6 * rv
        assert np.array_equal(np.sign(g), np.sign(rg))
        assert np.max(np.abs(g - rg)) <= 1e-7 * np.abs(rg).max()
    # the packed layout gives the same result
    lp, gp = R.loss_l1(cams, torch.tensor(np.concatenate(preds), device=DEV),
                       torch.tensor(np.concatenate(targets), device=DEV))
    assert np.array_equal(lp.cpu().numpy(), loss)
    assert np.array_equal(gp.cpu().numpy(), np.concatenate([g.cpu().numpy() for g in grads]))


def test_pose_adam_kernel():
    rng = np.random.default_rng(91)
    V, K = 3, 7
    poses = np.stack([S.random_pose_near_identity(92 + k, 10.0, 0.5) for k in range(V)])
    grads = rng.standard_normal((K, V, 6)).astype(np.float32)
    P = torch.tensor(poses, device=DEV)
    m = torch.zeros((V, 6), device=DEV)
    v = torch.zeros((V, 6), device=DEV)
    st = torch.zeros(V, dtype=torch.int32, device=DEV)
    ref = [(poses[k].astype(np.float64), np.zeros(6), np.zeros(6)) for k in range(V)]
    for it in range(K):
        R.pose_adam(P, torch.tensor(grads[it], device=DEV), m, v, st, 1e-2, 1e-3, K)
        frac = it / (K - 1)
        lr = 1e-3 + 0.5 * (1e-2 - 1e-3) * (1 + np.cos(np.pi * frac))
        ref = [oracle.pose_adam(T, mm, vv, grads[it][k], it + 1, lr)[:3] for k, (T, mm, vv) in enumerate(ref)]
    got = P.cpu().numpy()
    for k in range(V):
        assert np.max(np.abs(got[k] - ref[k][0])) <= 2e-6
    assert np.all(st.cpu().numpy() == K)
    # a guard workspace whose counters report an overflow skips the step
    guard = torch.zeros(64, dtype=torch.uint8, device=DEV)
    guard.view(torch.int32)[2] = 1
    before = [t.clone() for t in (P, m, v, st)]
    R.pose_adam(P, torch.tensor(grads[0], device=DEV), m, v, st, 1e-2, 1e-3, K, guard=guard)
    for a, b in zip(before, (P, m, v, st)):
        assert torch.equal(a, b)
    guard.zero_()
    R.pose_adam(P, torch.tensor(grads[0], device=DEV), m, v, st, 1e-2, 1e-3, K, guard=guard)
    assert np.all(st.cpu().numpy() == K + 1)


def test_autograd_function_matches_direct_calls():
    sc, cam, pose = random_case(101, 3, 64, 48, 300)
    g = R.GaussianParams.from_set(sc, DEV)
    params = [t.clone().requires_grad_(True) for t in (g.means, g.scales, g.quats, g.opacities, g.sh)]
    tau = torch.zeros((1, 6), device=DEV, requires_grad=True)
    P = torch.tensor(pose[None], device=DEV)
    W = torch.tensor(_upstream(102, cam).ravel(), device=DEV)
    img = R.render(g, [cam], P, tau=tau, params=params)
    (img * W).sum().backward()
    direct = _gpu(sc, [cam], [pose], up=[_upstream(102, cam)])
    assert np.array_equal(tau.grad.cpu().numpy(), direct["pose"])
    for t, k in zip(params, ("means", "scales", "quats", "opacities", "sh")):
        assert np.array_equal(t.grad.cpu().numpy(), direct[k])


def test_pose_solve_reduces_error_tiny():
    wl = S.tiny()
    cam = f32_camera(wl.camera)
    g = R.GaussianParams.from_set(wl.scene, DEV)
    target_pose = torch.tensor(wl.pose[None], device=DEV)
    rast = R.Rasterizer(0)
    target, _ = rast.forward(g, [cam], target_pose)
    target = target.clone()
    init = torch.tensor(wl.init_pose[None], device=DEV)
    est, hist = R.solve_poses(g, [cam], target, init, steps=150, lr=(1e-2, 1e-4), history=True)
    r0, t0 = S.pose_error(wl.init_pose, wl.pose)
    r1, t1 = S.pose_error(est[0].cpu().numpy(), wl.pose)
    print(f"tiny solve: rot {r0:.3f} -> {r1:.3f} deg, trans {t0:.4f} -> {t1:.4f}, loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    assert hist[-1] < 0.5 * hist[0]
    assert r1 < 0.5 * r0 and t1 < 0.5 * t0


def test_full_size_single_view_workload():
    """The benchmark workload at its full size (200k Gaussians, SH 3,
    1008x756): image, sort keys and gradients against the oracle."""
    wl = S.single_view()
    cam = f32_camera(wl.camera)
    sc, pose = wl.scene, wl.init_pose
    up = _upstream(111, cam)
    run = _gpu(sc, [cam], [pose], up=[up], want=())
    ref = oracle.render(sc, cam, pose)
    _image_check(run["images"][0], ref, "full-size")
    rref = oracle.backward(sc, cam, pose, up)
    rho = assert_grad_close(run["pose"][0, :3], rref["pose"][:3], "rho")
    phi = assert_grad_close(run["pose"][0, 3:], rref["pose"][3:], "phi")
    print(f"full-size pose gradient (rel L2, max element): rho {rho} phi {phi}")
    # the 2D splat gradients of every Gaussian, element by element; a
    # backward that wants no opacity gradient leaves that component zero
    g2 = run["rast"].inspect(run["g"], [cam], "grad2d").cpu().numpy().reshape(-1, 9)
    keep = [0, 1, 2, 3, 4, 6, 7, 8]
    assert_grad_close(g2[:, keep], rref["splat2d"][:, keep], "splat2d")
    assert np.all(g2[:, 5] == 0)
    # keys and values bit for bit (fragile Gaussians' instances excluded)
    sp = oracle.preprocess(sc, cam, pose)
    gw, gh = oracle.tiles_of(cam)
    rkeys, rvals = oracle.bin_sort([sp], [(gw, gh)])
    rast, g = run["rast"], run["g"]
    M, ovf = rast.instances()
    assert not ovf
    keys, vals = _sorted_instances(rast, g, [cam], M)
    fragile = np.nonzero(sp["fragile"])[0]
    print(f"full-size: M = {M}, fragile Gaussians {len(fragile)}")
    assert_sorted_match(keys, vals, rkeys, rvals, fragile)


def test_autograd_refuses_a_stale_forward():
    """A second render on the same Rasterizer overwrites the workspace the
    first render's backward needs: backpropagating the first then raises
    instead of returning the second render's gradients."""
    sc, cam, pose = random_case(103, 1, 48, 32, 200)
    g = R.GaussianParams.from_set(sc, DEV)
    params = [t.clone().requires_grad_(True) for t in (g.means, g.scales, g.quats, g.opacities, g.sh)]
    P = torch.tensor(pose[None], device=DEV)
    rast = R.Rasterizer(0)
    img1 = R.render(g, [cam], P, rast=rast, params=params)
    img2 = R.render(g, [cam], P, rast=rast, params=params)
    with pytest.raises(RuntimeError, match="rendered again"):
        img1.sum().backward()
    img2.sum().backward()      # the latest forward still back-propagates
    assert torch.isfinite(params[0].grad).all()


def _se3_hat(t):
    X = np.zeros((4, 4))
    r, p = t[:3], t[3:]
    X[:3, :3] = [[0, -p[2], p[1]], [p[2], 0, -p[0]], [-p[1], p[0], 0]]
    X[:3, 3] = r
    return X


def test_render_applies_a_nonzero_twist():
    """render() with a nonzero tau renders at Exp(tau) T and returns dL/dtau
    at that tau: the left twist gradient at the moved pose chained through
    the left Jacobian of SE(3), here taken by central differences of
    scipy's matrix exponential and logarithm."""
    import scipy.linalg as sl
    sc, cam, pose = random_case(104, 2, 64, 48, 400)
    g = R.GaussianParams.from_set(sc, DEV)
    tau0 = (np.random.default_rng(5).standard_normal(6) * 0.05).astype(np.float32)
    tau = torch.tensor(tau0[None], device=DEV, requires_grad=True)
    W = _upstream(105, cam)
    img = R.render(g, [cam], torch.tensor(pose[None], device=DEV), tau=tau)
    (img * torch.tensor(W.ravel(), device=DEV)).sum().backward()
    H = np.vstack([pose.astype(np.float64), [0, 0, 0, 1]])
    moved = (sl.expm(_se3_hat(tau0.astype(np.float64))) @ H)[:3].astype(np.float32)
    ref = _gpu(sc, [cam], [moved], up=[W])
    assert np.max(np.abs(img.detach().cpu().numpy().reshape(ref["images"][0].shape)
                         - ref["images"][0])) <= 1e-4
    E = sl.expm(_se3_hat(tau0.astype(np.float64)))
    Ei = np.linalg.inv(E)
    vee = lambda X: np.array([X[0, 3], X[1, 3], X[2, 3], X[2, 1], X[0, 2], X[1, 0]])
    J = np.zeros((6, 6))
    for j in range(6):
        d = np.zeros(6)
        d[j] = 1e-6
        Jp = vee(sl.logm(sl.expm(_se3_hat(tau0 + d)) @ Ei).real)
        Jm = vee(sl.logm(sl.expm(_se3_hat(tau0 - d)) @ Ei).real)
        J[:, j] = (Jp - Jm) / 2e-6
    expect = J.T @ ref["pose"][0].astype(np.float64)
    got = tau.grad.cpu().numpy()[0]
    print("tau grad", got, "expected", expect)
    assert rel_l2(got, expect) <= 1e-4
    assert rel_l2(got, ref["pose"][0]) > 1e-3    # the chain rule is not the identity here
