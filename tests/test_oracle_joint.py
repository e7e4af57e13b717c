"""Pins of the joint-objective oracle (oracle/joint.py) against mathematics
and libraries that are independent of it: scipy's Gaussian window and 2D
correlation, the adjoint identity, SSIM's closed forms on constant images
(inside and at a corner, where the zero padding shows), central finite
differences, and torch autograd + torch.optim.Adam for the Gaussian update."""
import numpy as np
import pytest
import scipy.signal
import torch

from oracle import joint as J


def test_window_matches_scipy():
    w = J.ssim_window()
    ref = scipy.signal.windows.gaussian(11, 1.5)
    assert np.max(np.abs(w - ref / ref.sum())) < 1e-15
    assert abs(w.sum() - 1) < 1e-15 and np.array_equal(w, w[::-1])


def test_filter_matches_scipy_correlate2d():
    rng = np.random.default_rng(1)
    w = J.ssim_window()
    w2 = np.outer(w, w)
    for H, W in ((7, 9), (13, 30), (24, 5)):
        img = rng.standard_normal((H, W))
        ref = scipy.signal.correlate2d(img, w2, mode="same", boundary="fill", fillvalue=0.0)
        assert np.max(np.abs(J._filter(img, w2) - ref)) < 1e-13


def test_filter_adjoint_identity():
    rng = np.random.default_rng(2)
    w2 = np.outer(J.ssim_window(), J.ssim_window())
    a = rng.standard_normal((12, 17))
    b = rng.standard_normal((12, 17))
    lhs = np.sum(J._filter(a, w2) * b)
    rhs = np.sum(a * J._filter_adjoint(b, w2))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_ssim_of_an_image_with_itself_is_one():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (3, 20, 23))
    assert np.max(np.abs(J.ssim_map(x, x) - 1)) < 1e-12
    val, grad = J.dssim(x, x)
    assert abs(val) < 1e-12 and np.max(np.abs(grad)) < 1e-12


def test_ssim_closed_form_on_constant_images():
    a, b = 0.7, 0.2
    x = np.full((1, 30, 30), a)
    y = np.full((1, 30, 30), b)
    s = J.ssim_map(x, y)[0]
    inner = (2 * a * b + J.SSIM_C1) / (a * a + b * b + J.SSIM_C1)   # all variances vanish
    # (the variances are differences E[x^2] - mu^2 whose rounding, ~1e-17,
    # is divided by C2 ~ 1e-3)
    assert abs(s[15, 15] - inner) < 1e-12
    # corner: the window keeps the mass c of its lower-right quarter
    w = J.ssim_window()
    c = w[5:].sum() ** 2
    mx, my = a * c, b * c
    sxx, syy, sxy = a * a * c - mx * mx, b * b * c - my * my, a * b * c - mx * my
    corner = ((2 * mx * my + J.SSIM_C1) * (2 * sxy + J.SSIM_C2)
              / ((mx * mx + my * my + J.SSIM_C1) * (sxx + syy + J.SSIM_C2)))
    assert abs(s[0, 0] - corner) < 1e-12


def test_ssim_is_symmetric():
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, (2, 14, 15))
    y = rng.uniform(0, 1, (2, 14, 15))
    assert np.max(np.abs(J.ssim_map(x, y) - J.ssim_map(y, x))) < 1e-14


@pytest.mark.parametrize("shape", [(3, 9, 12), (1, 16, 5)])
def test_dssim_gradient_by_central_differences(shape):
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, shape)
    y = np.clip(x + rng.normal(0, 0.2, shape), 0, 1)
    _, g = J.dssim(x, y)
    h = 1e-5
    fd = np.zeros_like(x)
    for idx in np.ndindex(*shape):
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd[idx] = (J.dssim(xp, y)[0] - J.dssim(xm, y)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-9 * max(1.0, np.max(np.abs(g)) * x.size)


def test_l1_and_rgb_loss():
    x = np.array([[[0.5, 0.2], [0.1, 0.9]]])
    y = np.array([[[0.5, 0.4], [0.0, 1.0]]])
    val, g = J.l1(x, y)
    assert abs(val - 0.4 / 4) < 1e-15
    assert np.array_equal(g, np.array([[[0.0, -0.25], [0.25, -0.25]]]))
    rng = np.random.default_rng(6)
    x = rng.uniform(0, 1, (3, 8, 8))
    y = rng.uniform(0, 1, (3, 8, 8))
    val, g = J.rgb_loss(x, y, 0.2)
    assert abs(val - (0.8 * J.l1(x, y)[0] + 0.2 * J.dssim(x, y)[0])) < 1e-15
    # no ties: the L1 part is smooth, finite differences hold for the sum
    h = 1e-6
    for idx in [(0, 0, 0), (1, 4, 3), (2, 7, 7)]:
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd = (J.rgb_loss(xp, y)[0] - J.rgb_loss(xm, y)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-8


def test_anisotropy_closed_forms():
    s = np.array([[1.0, 1.0, 20.0], [2.0, 3.0, 4.0], [0.5, 5.0, 0.5]])
    val, g = J.anisotropy(s, 10.0)
    # only the first Gaussian exceeds the ratio; the third sits exactly at r
    assert abs(val - (20.0 - 10.0) / 3) < 1e-15
    assert np.array_equal(g[1], np.zeros(3)) and np.array_equal(g[2], np.zeros(3))
    assert abs(g[0, 2] - 1.0 / 3) < 1e-15              # d/ds_max = 1 / (N s_min)
    assert abs(g[0, 0] + 20.0 / 3) < 1e-15             # d/ds_min = -s_max / (N s_min^2), first of the ties
    assert g[0, 1] == 0.0


def test_anisotropy_gradient_by_central_differences():
    rng = np.random.default_rng(7)
    s = np.exp(rng.uniform(-3, 1, (40, 3)))
    s[:10, 0] *= 50.0
    _, g = J.anisotropy(s, 10.0)
    h = 1e-7
    for i in range(40):
        for k in range(3):
            sp = s.copy(); sp[i, k] += h * s[i, k]
            sm = s.copy(); sm[i, k] -= h * s[i, k]
            fd = (J.anisotropy(sp)[0] - J.anisotropy(sm)[0]) / (2 * h * s[i, k])
            assert abs(fd - g[i, k]) < 1e-6 * max(1.0, abs(g[i, k]))


def _random_raw(rng, n, S):
    return {
        "means": rng.normal(0, 1, (n, 3)),
        "log_scales": rng.uniform(-4, -1, (n, 3)) + np.where(rng.random((n, 1)) < 0.3, [[3.0, 0, 0]], 0.0),
        "quats": rng.normal(0, 1, (n, 4)),
        "logit_opacities": rng.normal(0, 1.5, n),
        "sh": rng.normal(0, 0.3, (n, S, 3)),
    }


def test_gaussian_adam_matches_torch_autograd_and_adam():
    rng = np.random.default_rng(8)
    n, S, T = 50, 16, 30
    raw = _random_raw(rng, n, S)
    m = {k: np.zeros_like(a) for k, a in raw.items()}
    v = {k: np.zeros_like(a) for k, a in raw.items()}
    P = {k: torch.tensor(a, dtype=torch.float64, requires_grad=True) for k, a in raw.items()}
    lr0, lr1 = 1.6e-2, 1.6e-4
    opt = torch.optim.Adam([
        {"params": [P["means"]], "lr": lr0},
        {"params": [P["log_scales"]], "lr": 5e-3},
        {"params": [P["quats"]], "lr": 1e-3},
        {"params": [P["logit_opacities"]], "lr": 5e-2},
        {"params": [P["sh"]], "lr": 1.0},       # per-coefficient rates applied below
    ], betas=(0.9, 0.999), eps=1e-15)
    for step in range(1, 4):
        grads = {"means": rng.normal(0, 1e-3, (n, 3)), "scales": rng.normal(0, 1e-2, (n, 3)),
                 "quats": rng.normal(0, 1e-3, (n, 4)), "opacities": rng.normal(0, 1e-3, n),
                 "sh": rng.normal(0, 1e-3, (n, S, 3))}
        raw, m, v, l_an = J.gaussian_adam(raw, grads, m, v, step, T)
        # torch: the same objective's raw gradient by autograd, then Adam
        opt.zero_grad()
        s = torch.exp(P["log_scales"])
        o = torch.sigmoid(P["logit_opacities"])
        ratio = s.max(dim=1).values / s.min(dim=1).values
        lan = torch.clamp(ratio - 10.0, min=0).mean()
        lin = ((torch.tensor(grads["means"]) * P["means"]).sum()
               + (torch.tensor(grads["scales"]) * s).sum()
               + (torch.tensor(grads["quats"]) * P["quats"]).sum()
               + (torch.tensor(grads["opacities"]) * o).sum()
               + (torch.tensor(grads["sh"]) * P["sh"]).sum())
        assert abs(lan.item() - l_an) < 1e-12
        (lin + lan).backward()
        opt.param_groups[0]["lr"] = float(np.exp(np.log(lr0) * (1 - (step - 1) / (T - 1))
                                                 + np.log(lr1) * (step - 1) / (T - 1)))
        scale = torch.full((1, S, 1), 2.5e-3 / 20, dtype=torch.float64)
        scale[0, 0, 0] = 2.5e-3
        sh_before = P["sh"].detach().clone()
        opt.step()
        with torch.no_grad():   # per-coefficient rates: rescale the unit-rate step
            P["sh"].copy_(sh_before + (P["sh"] - sh_before) * scale)
        for k in J.GROUPS:
            ref = P[k].detach().numpy()
            assert np.max(np.abs(raw[k] - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref))), (k, step)


def test_gaussian_adam_first_step_is_signed_learning_rate():
    rng = np.random.default_rng(9)
    raw = _random_raw(rng, 20, 1)
    zeros = {k: np.zeros_like(a) for k, a in raw.items()}
    grads = {"means": rng.normal(0, 1, (20, 3)), "scales": np.zeros((20, 3)),
             "quats": rng.normal(0, 1, (20, 4)), "opacities": rng.normal(0, 1, 20),
             "sh": rng.normal(0, 1, (20, 1, 3))}
    new, _, _, _ = J.gaussian_adam(raw, grads, zeros, zeros, 1, 100, aniso_weight=0.0)
    assert np.allclose(new["means"] - raw["means"], -1.6e-2 * np.sign(grads["means"]), atol=1e-15)
    assert np.allclose(new["quats"] - raw["quats"], -1e-3 * np.sign(grads["quats"]), atol=1e-15)
    assert np.allclose(new["logit_opacities"] - raw["logit_opacities"],
                       -5e-2 * np.sign(grads["opacities"]), atol=1e-15)
    assert np.allclose(new["sh"] - raw["sh"], -2.5e-3 * np.sign(grads["sh"]), atol=1e-15)
    assert np.array_equal(new["log_scales"], raw["log_scales"])    # zero gradient, no L_An


def test_means_learning_rate_schedule():
    assert J.means_lr(1, 30, 1.6e-2, 1.6e-4) == pytest.approx(1.6e-2, rel=1e-15)
    assert J.means_lr(30, 30, 1.6e-2, 1.6e-4) == pytest.approx(1.6e-4, rel=1e-14)
    assert J.means_lr(15.5, 30, 1.6e-2, 1.6e-4) == pytest.approx(1.6e-3, rel=1e-14)   # geometric mean
    assert J.means_lr(99, 30, 1.6e-2, 1.6e-4) == pytest.approx(1.6e-4, rel=1e-14)
