"""gsp_render_bwd_pose_step, the pose-only backward whose final pose
reduction also applies the tangent-space Adam step (Sec. III-B), against the
two calls it replaces (gsp_render_bwd with the pose gradient only, then
gsp_pose_adam guarded by the same workspace): poses, gradients, moments and
step counts bit for bit over several iterations, in both pose
parametrisations, with two views per launch, and with an overflowing render
whose step must be skipped."""
import numpy as np
import pytest
import torch

from paper_2410_08743_amd import render as R
from paper_2410_08743_amd import synthetic as S
from tests.parity_util import random_case

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _setup(n_views):
    sc, cam, pose = random_case(71, 2, 96, 64, 600)
    cams = [cam] * n_views
    g = R.GaussianParams.from_set(sc, DEV)
    gt = torch.tensor(np.stack([pose] * n_views), device=DEV)
    init = torch.tensor(np.stack([S.perturb_pose(pose, 3.0, 0.08, S.rng_for(72 + v, 7))
                                  for v in range(n_views)]), dtype=torch.float32, device=DEV)
    target = R.Rasterizer(0).forward(g, cams, gt)[0].clone()
    return g, cams, target, init.contiguous()


def _solve(fused, g, cams, target, init, param, iters=6, capacity=None):
    rast = R.Rasterizer(0) if capacity is None else R.Rasterizer(0, capacity=capacity)
    V = len(cams)
    P = init.clone()
    m = torch.zeros((V, 6), device=DEV)
    v = torch.zeros((V, 6), device=DEV)
    st = torch.zeros(V, dtype=torch.int32, device=DEV)
    dpose = torch.zeros((V, 6), device=DEV)
    trace = []
    for _ in range(iters):
        _, dl, _ = rast.forward_l1(g, cams, P, target, check=False)
        if fused:
            rast.backward_pose_step(g, cams, P, dl, dpose, m, v, st, 1e-2, 1e-4, iters,
                                    parametrization=param)
        else:
            rast.backward(g, cams, P, dl, want=(), pose=True, out={"pose": dpose})
            R.pose_adam(P, dpose, m, v, st, 1e-2, 1e-4, iters, guard=rast.ws,
                        parametrization=param)
        trace.append([t.cpu().numpy().copy() for t in (P, dpose, m, v, st)])
    return trace, rast


@pytest.mark.parametrize("param", ["se3", "t_so3"])
@pytest.mark.parametrize("n_views", [1, 2])
def test_fused_pose_step_equals_backward_then_adam(param, n_views):
    g, cams, target, init = _setup(n_views)
    fused, _ = _solve(True, g, cams, target, init, param)
    split, _ = _solve(False, g, cams, target, init, param)
    for it, (a, b) in enumerate(zip(fused, split)):
        for name, x, y in zip(("poses", "dpose", "m", "v", "steps"), a, b):
            assert np.array_equal(x, y), f"iteration {it}: {name} differs"
    assert not np.array_equal(fused[-1][0], init.cpu().numpy())   # the poses moved
    assert (fused[-1][4] == len(fused)).all()


def test_fused_pose_step_skips_an_overflowed_render():
    g, cams, target, init = _setup(1)
    trace, rast = _solve(True, g, cams, target, init, "se3", iters=1, capacity=64)
    assert rast.instances()[1]   # the render overflowed its capacity
    P, _, m, v, st = trace[0]
    assert np.array_equal(P, init.cpu().numpy())
    assert not m.any() and not v.any() and not st.any()
