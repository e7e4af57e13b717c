"""The oracle's analytic gradient against a second, independent derivation:
forward-mode dual numbers through the whole render (oracle/dual.py), for
every parameter group and the pose twist, element by element.

The cases are chosen so that every branch of the derivative is exercised:
near-plane culling, Gaussians beyond the projection-Jacobian clamp, splats
clamped at alpha = 0.99 (zero derivative to opacity and power), colour
channels clamped at 0, pixels that stop at the 1e-4 transmittance bound, a
region of interest and a background colour.  Both derivations are FP64, so
they agree to rounding: 1e-12 of the group's largest entry per element."""
import numpy as np
import pytest

import oracle
from oracle import dual as D
from paper_2410_08743_amd import synthetic as S
from tests.parity_util import random_case

GROUPS = ("means", "scales", "quats", "opacities", "sh")


def _case(name):
    if name == "sh0-near-clamp":
        # depths down to the near plane and lateral spread beyond the J clamp
        sc, cam, pose = random_case(3, 0, 40, 36, 12, depth=(0.1, 4.0), lateral=1.6)
        # two Gaussians in front of the near plane (camera frame z = 0.15, 0.19)
        R, t = pose[:, :3].astype(np.float64), pose[:, 3].astype(np.float64)
        for i, z in ((0, 0.15), (1, 0.19)):
            sc.means[i] = (R.T @ (np.array([0.02, -0.01, z]) - t)).astype(np.float32)
        return sc, cam, pose
    if name == "sh3-roi-bg":
        sc, cam, pose = random_case(5, 3, 80, 64, 14, roi=(16, 16, 40, 30), depth=(0.5, 5.0))
        return sc, cam, pose
    if name == "sh1-saturating":
        # opaque, large splats: alpha clamped at 0.99 and the 1e-4 stop
        sc, cam, pose = random_case(7, 1, 36, 34, 60, depth=(1.0, 4.0), lateral=0.4)
        sc.opacities[:] = np.float32(0.9999)
        sc.scales[:] = np.float32([0.3, 0.2, 0.12])
        return sc, cam, pose
    if name == "sh2-dark":
        # negative DC terms: colour channels clamped at 0
        sc, cam, pose = random_case(9, 2, 34, 40, 12, depth=(0.8, 4.0), lateral=1.0)
        sc.sh[::2, 0, 1] = np.float32(-3.0)
        return sc, cam, pose
    raise KeyError(name)


CASES = ["sh0-near-clamp", "sh3-roi-bg", "sh1-saturating", "sh2-dark"]


def _events(sc, cam, pose):
    sp = oracle.preprocess(sc, cam, pose)
    x, y, w, h = cam.region()
    clamped_alpha = stopped = 0
    for py in range(y, y + h):
        for px in range(x, x + w):
            tr = oracle.pixel_trace(sc, cam, pose, px, py)
            clamped_alpha += int(np.sum(tr["alpha_clamped"] & tr["blended"]))
            stopped += int(len(tr) > 0 and not tr[-1]["blended"] and tr[-1]["alpha"] >= 1 / 255)
    return {
        "culled": int(np.sum(sp["p"][:, 2] <= 0.2)),
        "jclamp": int(np.sum(sp["jclamp"].any(1) & (sp["rendered"] == 1))),
        "color_clamped": int(np.sum(sp["color_clamped"].any(1) & (sp["rendered"] == 1))),
        "alpha_clamped": clamped_alpha,
        "stopped": stopped,
    }


@pytest.mark.parametrize("name", CASES)
def test_analytic_gradient_equals_dual_numbers(name):
    sc, cam, pose = _case(name)
    x, y, w, h = cam.region()
    Wt = np.random.default_rng(len(name)).standard_normal((3, h, w))
    val, g = D.gradient_of_linear_loss(sc, cam, pose, Wt)
    ref = oracle.render(sc, cam, pose)
    assert np.max(np.abs(val - ref["image"])) <= 1e-13   # same render, same decisions
    back = oracle.backward(sc, cam, pose, Wt)
    for k in GROUPS:
        scale = max(np.abs(back[k]).max(), 1e-300)
        err = np.abs(g[k] - back[k]).max() / scale
        assert err <= 1e-12, (k, err)
    for sl, k in ((slice(0, 3), "rho"), (slice(3, 6), "phi")):
        err = np.abs(g["pose"][sl] - back["pose"][sl]).max() / np.abs(back["pose"][sl]).max()
        assert err <= 1e-12, (k, err)


def test_cases_cover_every_branch():
    seen = {}
    for name in CASES:
        ev = _events(*_case(name))
        print(name, ev)
        for k, v in ev.items():
            seen[k] = seen.get(k, 0) + v
    assert all(v > 0 for v in seen.values()), seen


def test_dual_numbers_detect_a_dropped_term():
    """The comparison has teeth: dropping the colour's dependence on the
    viewing direction (a plausible slip in the SH chain rule) moves the
    mean and pose gradients far beyond the bar."""
    sc, cam, pose = _case("sh3-roi-bg")
    x, y, w, h = cam.region()
    Wt = np.random.default_rng(1).standard_normal((3, h, w))
    keep = D._sh_basis
    try:
        def frozen(deg, x_, y_, z_):
            return [D.Dual(e.v, e.d * 0.0) for e in keep(deg, x_, y_, z_)]
        D._sh_basis = frozen
        _, g = D.gradient_of_linear_loss(sc, cam, pose, Wt)
    finally:
        D._sh_basis = keep
    back = oracle.backward(sc, cam, pose, Wt)
    err = np.abs(g["means"] - back["means"]).max() / np.abs(back["means"]).max()
    assert err > 1e-6
