"""Stored-list mode (the forward keeps every pixel's blended entries with
their alpha and the transmittance in front of them; the backward reads them)
against the recomputing backward and against the oracle, through the C ABI.

Bars: images bit-identical (the forward is the same); the stored pairs are
exactly the forward's blended (pixel, splat) pairs (their count equals the
forward's own per-pixel blend counts); gradients of the two backward modes
within 1e-5 relative L2 per group (the recomputing walk divides its way back
to T_i, the stored one reads T_i: they differ by FP32 rounding of that
recovery only, which 1 - alpha >= 0.01 keeps bounded); stored-mode
gradients against the oracle as for the default backward."""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_08743_amd import render as R
from tests.parity_util import assert_grad_close, max_rel_inf, rel_l2
from tests.test_gpu_parity import CASES, _case, _upstream

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NAMES = ("means", "scales", "quats", "opacities", "sh")


def _run(sc, cams, poses, ups, store, pair_capacity=0):
    g = R.GaussianParams.from_set(sc, DEV)
    P = torch.tensor(np.stack(poses), device=DEV, dtype=torch.float32)
    rast = R.Rasterizer(0, store_lists=store, pair_capacity=pair_capacity)
    img, _ = rast.forward(g, cams, P)
    dl = torch.tensor(np.concatenate([u.ravel() for u in ups]), device=DEV)
    gr = rast.backward(g, cams, P, dl)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in gr.items()}
    out["image"] = img.cpu().numpy()
    out["grad2d"] = rast.inspect(g, cams, "grad2d").cpu().numpy()
    out["rast"], out["g"] = rast, g
    return out


@pytest.mark.parametrize("name", CASES)
def test_stored_lists_match_recompute_and_oracle(name):
    sc, cam, pose = _case(name)
    up = _upstream(21, cam)
    rec = _run(sc, [cam], [pose], [up], store=False)
    sto = _run(sc, [cam], [pose], [up], store=True)
    assert np.array_equal(rec["image"], sto["image"])
    q, ovf = sto["rast"].list_pairs()
    assert not ovf
    # the stored pairs are the forward's blended pairs: same count as the
    # forward's own per-pixel blend counters
    R.profile_enable(0, R.PROFILE_COUNTS)
    try:
        r2 = R.Rasterizer(0)
        r2.forward(rec["g"], [cam], torch.tensor(pose[None], device=DEV))
        nb = r2.inspect(rec["g"], [cam], "nblend", torch.int32).cpu().numpy().astype(np.int64)
    finally:
        R.profile_enable(0, 0)
    assert q == int(nb.sum()), (q, int(nb.sum()))
    report = {}
    for k in NAMES + ("grad2d",):
        report[k] = (rel_l2(sto[k], rec[k]), max_rel_inf(sto[k], rec[k]))
        assert_grad_close(sto[k], rec[k], f"stored vs recompute {k}", rel=1e-5, elem=1e-4)
    for sl, k in ((slice(0, 3), "rho"), (slice(3, 6), "phi")):
        report[k] = (rel_l2(sto["pose"][0, sl], rec["pose"][0, sl]),)
        assert_grad_close(sto["pose"][0, sl], rec["pose"][0, sl], f"stored vs recompute {k}",
                          rel=1e-5, elem=1e-5)
    print(name, f"pairs {q}", {k: tuple(f"{x:.1e}" for x in v) for k, v in report.items()})
    ref = oracle.backward(sc, cam, pose, up)
    for k in NAMES:
        assert_grad_close(sto[k], ref[k], f"stored vs oracle {k}")
    assert_grad_close(sto["pose"][0, :3], ref["pose"][:3], "stored vs oracle rho")
    assert_grad_close(sto["pose"][0, 3:], ref["pose"][3:], "stored vs oracle phi")


def test_stored_lists_batched_views_equal_single_views():
    from tests.parity_util import f32_camera, random_case
    from paper_2410_08743_amd import synthetic as S
    sc, cam0, pose0 = random_case(31, 3, 96, 64, 800)
    cam1 = f32_camera(S.Camera(80, 48, 75.0, 70.0, 40.5, 23.75, roi=(16, 0, 50, 48)))
    pose1 = S.random_pose_near_identity(32, 3.0, 0.1)
    cams, poses = [cam0, cam1], [pose0, pose1]
    ups = [_upstream(40 + k, c) for k, c in enumerate(cams)]
    both = _run(sc, cams, poses, ups, store=True)
    for k in range(2):
        one = _run(sc, [cams[k]], [poses[k]], [ups[k]], store=True)
        assert np.array_equal(both["pose"][k], one["pose"][0])


def test_pair_capacity_overflow_is_reported_and_regrown():
    sc, cam, pose = _case("sh3-dense")
    up = _upstream(22, cam)
    full = _run(sc, [cam], [pose], [up], store=True)
    need, _ = full["rast"].list_pairs()
    g = full["g"]
    P = torch.tensor(pose[None], device=DEV)
    rast = R.Rasterizer(0, store_lists=True, pair_capacity=need // 3)
    rast.forward(g, [cam], P, check=False)
    q, ovf = rast.list_pairs()
    assert ovf and q == need
    dl = torch.tensor(up.ravel(), device=DEV)
    gr = rast.backward(g, [cam], P, dl)      # of an overflowed forward: zero gradients
    torch.cuda.synchronize()
    assert float(gr["means"].abs().max()) == 0.0 and float(gr["pose"].abs().max()) == 0.0
    assert rast.overflowed()
    rast.lists = None                        # regrow on the next checked forward
    rast.forward(g, [cam], P, check=True)
    assert rast.pair_capacity >= need and not rast.list_pairs()[1]
    gr = rast.backward(g, [cam], P, dl)
    assert np.array_equal(gr["means"].cpu().numpy(), full["means"])
    assert np.array_equal(gr["pose"].cpu().numpy(), full["pose"])


def test_autograd_function_with_stored_lists():
    sc, cam, pose = _case("sh1-ragged")
    up = _upstream(23, cam)
    direct = _run(sc, [cam], [pose], [up], store=True)
    g = R.GaussianParams.from_set(sc, DEV)
    params = [t.clone().requires_grad_(True) for t in (g.means, g.scales, g.quats, g.opacities, g.sh)]
    tau = torch.zeros((1, 6), device=DEV, requires_grad=True)
    rast = R.Rasterizer(0, store_lists=True)
    img = R.render(g, [cam], torch.tensor(pose[None], device=DEV), tau=tau, rast=rast, params=params)
    (img * torch.tensor(up.ravel(), device=DEV)).sum().backward()
    assert np.array_equal(tau.grad.cpu().numpy(), direct["pose"])
    for t, k in zip(params, NAMES):
        assert np.array_equal(t.grad.cpu().numpy(), direct[k])
