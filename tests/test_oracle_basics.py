"""Pins of the oracle's building blocks against mathematics and libraries
that are independent of it: SH orthonormality by quadrature and the complex
spherical harmonics of scipy, quaternion rotations of scipy, the matrix
exponential of scipy, torch's Adam, and the plain definition of L1."""
import numpy as np
import pytest
import scipy.linalg
import scipy.special
from scipy.spatial.transform import Rotation

import oracle


def _complex_sh(l, m, d):
    """scipy's complex Y_l^m (Condon-Shortley phase) at unit direction d."""
    x, y, z = d
    theta = np.arccos(np.clip(z, -1, 1))          # polar
    phi = np.arctan2(y, x)                         # azimuth
    if hasattr(scipy.special, "sph_harm_y"):
        return scipy.special.sph_harm_y(l, m, theta, phi)
    return scipy.special.sph_harm(m, l, phi, theta)


def _real_sh_reference(degree, d):
    """Real basis from the complex one: sqrt(2) Im Y_l^|m| for m < 0, Y_l^0,
    sqrt(2) Re Y_l^m for m > 0, ordered m = -l..l."""
    out = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            if m < 0:
                out.append(np.sqrt(2.0) * _complex_sh(l, -m, d).imag)
            elif m == 0:
                out.append(_complex_sh(l, 0, d).real)
            else:
                out.append(np.sqrt(2.0) * _complex_sh(l, m, d).real)
    return np.array(out)


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform azimuth: exact for the degree-6
    # polynomials that products of degree-3 harmonics are.
    zs, wz = np.polynomial.legendre.leggauss(8)
    nphi = 16
    phis = 2 * np.pi * np.arange(nphi) / nphi
    gram = np.zeros((16, 16))
    for z, w in zip(zs, wz):
        r = np.sqrt(1 - z * z)
        for ph in phis:
            d = np.array([r * np.cos(ph), r * np.sin(ph), z])
            Y = oracle.sh_basis(3, d)
            gram += np.outer(Y, Y) * w * (2 * np.pi / nphi)
    assert np.max(np.abs(gram - np.eye(16))) < 1e-12


def test_sh_matches_scipy_complex_harmonics():
    rng = np.random.default_rng(5)
    for _ in range(50):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        ref = _real_sh_reference(3, d)
        got = oracle.sh_basis(3, d)
        assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_sh_lower_degrees_are_prefixes(degree):
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    full = oracle.sh_basis(3, d)
    assert np.array_equal(oracle.sh_basis(degree, d), full[: (degree + 1) ** 2])


def test_sh_gradient_by_central_differences():
    rng = np.random.default_rng(6)
    for _ in range(20):
        d = rng.standard_normal(3)
        _, G = oracle.sh_basis(3, d, with_grad=True)
        h = 1e-6
        fd = np.zeros((16, 3))
        for e in range(3):
            dp, dm = d.copy(), d.copy()
            dp[e] += h
            dm[e] -= h
            fd[:, e] = (oracle.sh_basis(3, dp) - oracle.sh_basis(3, dm)) / (2 * h)
        assert np.max(np.abs(fd - G)) < 1e-7 * max(1.0, np.max(np.abs(G)))


def test_quaternion_rotation_matches_scipy():
    rng = np.random.default_rng(7)
    for _ in range(100):
        q = rng.standard_normal(4) * rng.uniform(0.1, 10.0)
        R = oracle.quat_to_rotmat(q)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()  # scipy: (x,y,z,w)
        assert np.max(np.abs(R - ref)) < 1e-14


def _hat(tau):
    rho, phi = tau[:3], tau[3:]
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]]
    X[:3, 3] = rho
    return X


@pytest.mark.parametrize("scale", [1e-7, 1e-5, 1e-3, 0.3, 2.5])
def test_se3_exp_matches_expm(scale):
    rng = np.random.default_rng(int(scale * 1e7) % 1000)
    for _ in range(20):
        tau = rng.standard_normal(6) * scale
        T = oracle.se3_exp(tau)
        ref = scipy.linalg.expm(_hat(tau))[:3, :]
        assert np.max(np.abs(T - ref)) < 1e-12


def test_se3_retract_is_left_composition():
    rng = np.random.default_rng(8)
    T0 = np.concatenate([Rotation.random(random_state=3).as_matrix(), rng.standard_normal((3, 1))], 1)
    d = rng.standard_normal(6) * 0.1
    got = oracle.se3_retract(d, T0)
    E = scipy.linalg.expm(_hat(d))
    ref = (E @ np.vstack([T0, [0, 0, 0, 1]]))[:3]
    assert np.max(np.abs(got - ref)) < 1e-12


def test_pose_adam_increments_match_torch_adam():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    grads = rng.standard_normal((12, 6))
    lrs = np.linspace(1e-2, 1e-3, 12)
    x = torch.zeros(6, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([x], lr=1.0, betas=(0.9, 0.999), eps=1e-8)
    T = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)
    m = np.zeros(6)
    v = np.zeros(6)
    for k in range(12):
        before = x.detach().clone()
        for gparam in opt.param_groups:
            gparam["lr"] = float(lrs[k])
        x.grad = torch.tensor(grads[k])
        opt.step()
        inc = (x.detach() - before).numpy()
        T_new, m, v, delta = oracle.pose_adam(T, m, v, grads[k], k + 1, lrs[k])
        assert np.max(np.abs(delta - inc)) < 1e-15 + 1e-12 * np.max(np.abs(inc))
        ref = (scipy.linalg.expm(_hat(delta)) @ np.vstack([T, [0, 0, 0, 1]]))[:3]
        assert np.max(np.abs(T_new - ref)) < 1e-12
        T = T_new


def test_l1_definition():
    rng = np.random.default_rng(10)
    a = rng.standard_normal(1000)
    b = a.copy()
    b[::3] += rng.standard_normal(334)
    val, grad = oracle.l1(a, b)
    assert abs(val - np.mean(np.abs(a - b))) < 1e-14
    assert np.array_equal(grad, np.sign(a - b) / a.size)
    assert np.all(grad[1::3][(a - b)[1::3] == 0] == 0)


def _stack_at_pixel(opacities):
    """Gaussians one behind the other on the optical axis of a 16 x 16
    camera whose pixel (8, 8) they hit dead centre (power = 0 there, so
    alpha = min(0.99, o) exactly), front to back in the given order."""
    from paper_2410_08743_amd import synthetic as S
    n = len(opacities)
    means = np.zeros((n, 3), np.float32)
    means[:, 2] = 1.0 + 0.25 * np.arange(n)
    sc = S.GaussianSet(means, np.full((n, 3), 0.05, np.float32),
                       np.tile(np.float32([1, 0, 0, 0]), (n, 1)),
                       np.asarray(opacities, np.float32), np.zeros((n, 1, 3), np.float32), 0)
    cam = S.Camera(16, 16, 16.0, 16.0, 8.5, 8.5)
    pose = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)
    return sc, cam, pose


# (front-to-back opacities, the accumulated opacity sum_i alpha_i T_i of the
# centre pixel worked out by hand, the mask of Eq. (20) for it)
_MASK_CASES = [
    ([0.5], 0.5, 0),
    # one splat clamped at alpha = 0.99: the sum is exactly 0.99, which is not
    # above the threshold (a ">=" reading would set the mask)
    ([0.99], 0.99, 0),
    # 0.99 in front, then alpha = 0.01 (float32) behind: 0.99 + 0.01 a2 > 0.99
    ([0.99, 0.01], 0.99 + 0.01 * float(np.float32(0.01)), 1),
    # six and seven halvings: 63/64 (below) and 127/128 (above), exact
    ([0.5] * 6, 63 / 64, 0),
    ([0.5] * 7, 127 / 128, 1),
]


def test_masked_l1_mask_at_the_threshold():
    """Eq. (20)-(21) on hand-computed pixels around the 0.99 threshold.  The
    accumulated opacity is read from the compositing trace itself (the sum of
    the blended weights alpha_i T_i, the quantity Eq. (20) thresholds), and
    the masked L1 is checked on residuals whose masked sum is known."""
    T_final, weights = [], []
    for opac, acc, _ in _MASK_CASES:
        sc, cam, pose = _stack_at_pixel(opac)
        tr = oracle.pixel_trace(sc, cam, pose, 8, 8)
        bl = tr[tr["blended"] == 1]
        assert len(bl) == len(opac)
        w = float(np.sum(bl["alpha"] * bl["T_before"]))
        assert abs(w - acc) <= 1e-15, (opac, w, acc)
        Tf = oracle.render(sc, cam, pose)["T_final"][8, 8]
        assert abs((1.0 - Tf) - w) <= 1e-15
        T_final.append(Tf)
        weights.append(w)
    assert weights[1] == 0.99      # exactly at the threshold
    mask = np.array([m for _, _, m in _MASK_CASES])
    # residuals r = a - b per pixel and channel, sum of |r| over the masked
    # pixels (2 and 4): |-0.5| + 0.25 + 0 + 2 + |-0.125| + 1 = 3.875
    r = np.array([[1.0, -0.5, -0.5, 3.0, 2.0],
                  [-2.0, 0.25, 0.25, 1.0, -0.125],
                  [0.5, 4.0, 0.0, -1.0, 1.0]])
    b = np.arange(15, dtype=np.float64).reshape(3, 5) / 8
    val, grad = oracle.masked_l1(b + r, b, np.array(T_final))
    assert val == 3.875
    assert np.array_equal(grad, np.sign(r) * mask[None])
    assert np.array_equal(grad[:, 0], np.zeros(3)) and np.array_equal(grad[:, 1], np.zeros(3))
    assert np.array_equal(grad[:, 2], [-1.0, 1.0, 0.0])


def test_masked_l1_definition():
    rng = np.random.default_rng(11)
    h, w = 20, 30
    a = rng.standard_normal((3, h, w))
    b = rng.standard_normal((3, h, w))
    T = rng.uniform(0, 0.03, (h, w))
    val, grad = oracle.masked_l1(a, b, T)
    mask = (1.0 - T) > 0.99
    assert abs(val - np.sum(np.abs(a - b) * mask[None])) < 1e-12
    assert np.array_equal(grad, np.sign(a - b) * mask[None])
