"""FP64 oracle of the joint reconstruction and pose refinement objective and
of the Gaussian parameter update (Sec. III-C).

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module.  numpy only; it imports
nothing from the product package and shares no code with the HIP library.

What it computes, in the paper's terms:
  L = L_RGB + L_An                                   (Eq. (15))
  L_RGB = (1 - beta) L_L1 + beta L_DSSIM, beta = 0.2 (Eq. (16))
  L_An = (1/N) sum_i [max(s_i) / min(s_i) - r]_+     (Eq. (17)), r = 10

Readings where the paper defers to 3DGS or is silent (each is also listed
with the design notes):
  * L_DSSIM = 1 - mean SSIM over the three channels and every pixel; SSIM is
    the local statistic with an 11 x 11 Gaussian window of sigma 1.5
    (normalised), C1 = 0.01^2, C2 = 0.03^2, evaluated at every pixel of the
    image with zero padding outside it (a 'same'-size filter).
  * L_L1 = mean |pred - target| over 3 x H x W; its derivative at equality
    is 0.
  * With several views in a step the losses of the views are summed, each a
    mean over its own pixels.
  * max / min over the three activated scales; where several scales tie,
    the first one in index order is the max (or min) that the derivative
    goes to; at ratio == r exactly the hinge's derivative is 0.
  * The Gaussian parameters are optimised in the 3DGS parametrisation:
    means, log scales, raw quaternions, logit opacities and SH coefficients;
    scales = exp(log scales), opacities = sigmoid(logits).  Adam per scalar
    with bias correction; the means' learning rate decays log-linearly
    (exponentially) from lr_means[0] at the first step to lr_means[1] at
    step total_steps, the other groups keep constant rates.
"""
import numpy as np

SSIM_SIZE = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window(size=SSIM_SIZE, sigma=SSIM_SIGMA):
    """Normalised 1D Gaussian window of the SSIM in the DSSIM term of
    Eq. (16); the 2D window is its outer product."""
    k = np.arange(size, dtype=np.float64) - (size // 2)
    w = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return w / w.sum()


def _filter(img, w2):
    """out[y, x] = sum_{a, b} w2[a, b] img[y + a - h, x + b - h] over the
    offsets whose pixel lies inside the image (zero padding)."""
    H, W = img.shape
    h = w2.shape[0] // 2
    out = np.zeros((H, W))
    for a in range(w2.shape[0]):
        for b in range(w2.shape[1]):
            dy, dx = a - h, b - h
            ys, ye = max(0, -dy), min(H, H - dy)
            xs, xe = max(0, -dx), min(W, W - dx)
            if ys >= ye or xs >= xe:
                continue
            out[ys:ye, xs:xe] += w2[a, b] * img[ys + dy:ye + dy, xs + dx:xe + dx]
    return out


def _filter_adjoint(g, w2):
    """Adjoint of _filter: out[q] = sum over the pixels p whose window holds q
    of w2[q - p + h] g[p]."""
    H, W = g.shape
    h = w2.shape[0] // 2
    out = np.zeros((H, W))
    for a in range(w2.shape[0]):
        for b in range(w2.shape[1]):
            dy, dx = a - h, b - h
            ys, ye = max(0, -dy), min(H, H - dy)
            xs, xe = max(0, -dx), min(W, W - dx)
            if ys >= ye or xs >= xe:
                continue
            out[ys + dy:ye + dy, xs + dx:xe + dx] += w2[a, b] * g[ys:ye, xs:xe]
    return out


def _moments(x, y, w2):
    mx, my = _filter(x, w2), _filter(y, w2)
    exx, eyy, exy = _filter(x * x, w2), _filter(y * y, w2), _filter(x * y, w2)
    return mx, my, exx - mx * mx, eyy - my * my, exy - mx * my


def ssim_map(x, y):
    """SSIM at every pixel of each channel (the DSSIM term of Eq. (16));
    x, y: [C, H, W]."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = ssim_window()
    w2 = np.outer(w, w)
    out = np.zeros_like(x)
    for c in range(x.shape[0]):
        mx, my, sxx, syy, sxy = _moments(x[c], y[c], w2)
        num = (2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)
        den = (mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2)
        out[c] = num / den
    return out


def dssim(x, y):
    """L_DSSIM of Eq. (16): (1 - mean SSIM, its gradient with respect to x)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = ssim_window()
    w2 = np.outer(w, w)
    n = x.size
    total = 0.0
    grad = np.zeros_like(x)
    for c in range(x.shape[0]):
        mx, my, sxx, syy, sxy = _moments(x[c], y[c], w2)
        a1 = 2 * mx * my + SSIM_C1
        a2 = 2 * sxy + SSIM_C2
        b1 = mx * mx + my * my + SSIM_C1
        b2 = sxx + syy + SSIM_C2
        s = a1 * a2 / (b1 * b2)
        total += s.sum()
        # partial derivatives of s in (mu_x, sigma_x^2, sigma_xy)
        ds_dmx = 2 * my * a2 / (b1 * b2) - 2 * mx * s / b1
        ds_dsxx = -s / b2
        ds_dsxy = 2 * a1 / (b1 * b2)
        # through sigma_x^2 = E[x^2] - mu_x^2 and sigma_xy = E[xy] - mu_x mu_y
        g_mean = ds_dmx - 2 * mx * ds_dsxx - my * ds_dsxy
        g_exx = ds_dsxx
        g_exy = ds_dsxy
        dsum = (_filter_adjoint(g_mean, w2) + 2 * x[c] * _filter_adjoint(g_exx, w2)
                + y[c] * _filter_adjoint(g_exy, w2))
        grad[c] = -dsum / n
    return 1.0 - total / n, grad


def l1(x, y):
    """L_L1 of Eq. (16): (mean |x - y|, its gradient; 0 where equal)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return np.abs(x - y).mean(), np.sign(x - y) / x.size


def rgb_loss(x, y, beta=0.2):
    """L_RGB of one view (Eq. (16)) and its gradient with respect to x."""
    a, ga = l1(x, y)
    b, gb = dssim(x, y)
    return (1 - beta) * a + beta * b, (1 - beta) * ga + beta * gb


def anisotropy(scales, r=10.0):
    """L_An (Eq. (17)) of activated scales [N, 3] and its gradient."""
    s = np.asarray(scales, dtype=np.float64)
    n = s.shape[0]
    grad = np.zeros_like(s)
    if n == 0:
        return 0.0, grad
    imax = np.argmax(s, axis=1)
    imin = np.argmin(s, axis=1)
    rows = np.arange(n)
    smax, smin = s[rows, imax], s[rows, imin]
    ratio = smax / smin
    active = ratio > r
    val = np.where(active, ratio - r, 0.0).sum() / n
    g_max = np.where(active, 1.0 / smin, 0.0) / n
    g_min = np.where(active, -smax / (smin * smin), 0.0) / n
    np.add.at(grad, (rows, imax), g_max)
    np.add.at(grad, (rows, imin), g_min)
    return val, grad


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def means_lr(step, total_steps, lr_start, lr_end):
    """The means' learning rate of Sec. IV-A (exponential decay): log-linear
    from lr_start at step 1 to lr_end at step total_steps."""
    if total_steps <= 1:
        return lr_start
    t = min(step - 1, total_steps - 1) / (total_steps - 1)
    return float(np.exp(np.log(lr_start) * (1 - t) + np.log(lr_end) * t))


GROUPS = ("means", "log_scales", "quats", "logit_opacities", "sh")


def gaussian_adam(raw, grads, m, v, step, total_steps, lr_means=(1.6e-2, 1.6e-4),
                  lr_sh_dc=2.5e-3, lr_sh_rest=2.5e-3 / 20, lr_opacity=5e-2, lr_scales=5e-3,
                  lr_quats=1e-3, beta1=0.9, beta2=0.999, eps=1e-15, aniso_r=10.0,
                  aniso_weight=1.0):
    """One Adam step on the raw Gaussian parameters, for the objective
    L = L_RGB + L_An of Eq. (15) (Sec. III-C; rates of Sec. IV-A).

    raw:   dict GROUPS -> arrays ([N,3], [N,3], [N,4], [N], [N,S,3])
    grads: dict of the gradients with respect to the ACTIVATED parameters
           ('means', 'scales', 'quats', 'opacities', 'sh'), as the renderer's
           backward gives them (quats: the raw quaternion)
    m, v:  dicts like raw (first and second moments); step: 1-based.
    The L_An term (weight aniso_weight) is added to the scale gradient.
    Returns (new raw, new m, new v, L_An of the parameters before the step).
    """
    s = np.exp(np.asarray(raw["log_scales"], dtype=np.float64))
    o = sigmoid(np.asarray(raw["logit_opacities"], dtype=np.float64))
    l_an, g_an = anisotropy(s, aniso_r)
    g = {
        "means": np.asarray(grads["means"], dtype=np.float64),
        "log_scales": (np.asarray(grads["scales"], dtype=np.float64) + aniso_weight * g_an) * s,
        "quats": np.asarray(grads["quats"], dtype=np.float64),
        "logit_opacities": np.asarray(grads["opacities"], dtype=np.float64) * o * (1 - o),
        "sh": np.asarray(grads["sh"], dtype=np.float64),
    }
    lr_sh = np.full(np.asarray(raw["sh"]).shape[1], lr_sh_rest)
    lr_sh[0] = lr_sh_dc
    lrs = {
        "means": means_lr(step, total_steps, *lr_means),
        "log_scales": lr_scales,
        "quats": lr_quats,
        "logit_opacities": lr_opacity,
        "sh": lr_sh[None, :, None],
    }
    c1 = 1 - beta1 ** step
    c2 = 1 - beta2 ** step
    new_raw, new_m, new_v = {}, {}, {}
    for k in GROUPS:
        mm = beta1 * np.asarray(m[k], dtype=np.float64) + (1 - beta1) * g[k]
        vv = beta2 * np.asarray(v[k], dtype=np.float64) + (1 - beta2) * g[k] * g[k]
        new_raw[k] = np.asarray(raw[k], dtype=np.float64) - lrs[k] * (mm / c1) / (np.sqrt(vv / c2) + eps)
        new_m[k] = mm
        new_v[k] = vv
    return new_raw, new_m, new_v, l_an
