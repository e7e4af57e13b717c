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
