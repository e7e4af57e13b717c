"""FP64 oracle of the decoupled pose parametrisation T x SO(3) that the
paper names as the alternative to its SE(3) poses (Sec. IV-A, left to
future work): the camera centre c in R^3 and the rotation R in SO(3) are
updated separately.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module.  numpy only; it imports
nothing from the product package and shares no code with the HIP library.

Given the left-twist gradient (dL/drho, dL/dphi) of a world->camera pose
T = [R | t] (the renderer's pose gradient), the gradient in (c, phi) with
c = -R^T t is dL/dc = -R^T dL/drho and dL/dphi unchanged (a left rotation
of T keeps the camera centre); Adam runs on that 6-vector, and the step is
c <- c + delta_c, R <- Exp(delta_phi) R, t = -R c.
"""
import numpy as np


def so3_exp(phi):
    """Rodrigues' formula: the SO(3) exponential of the rotation update."""
    phi = np.asarray(phi, dtype=np.float64)
    th = np.linalg.norm(phi)
    K = np.array([[0.0, -phi[2], phi[1]], [phi[2], 0.0, -phi[0]], [-phi[1], phi[0], 0.0]])
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * (K @ K)


def txso3_gradient(pose, g):
    """(dL/dc, dL/dphi) from the left-twist gradient g = (rho, phi) of
    Sec. III-B (Eq. (7)-(13)), for the T x SO(3) alternative of Sec. IV-A."""
    R = np.asarray(pose, dtype=np.float64)[:, :3]
    g = np.asarray(g, dtype=np.float64)
    return np.concatenate([-R.T @ g[:3], g[3:]])


def pose_adam_txso3(pose, m, v, g, k, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """(new pose [3, 4], m, v, delta) after the k-th (1-based) T x SO(3)
    Adam step with left-twist gradient g."""
    pose = np.asarray(pose, dtype=np.float64)
    R, t = pose[:, :3], pose[:, 3]
    gg = txso3_gradient(pose, g)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * gg
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * gg * gg
    delta = -lr * (m / (1 - beta1 ** k)) / (np.sqrt(v / (1 - beta2 ** k)) + eps)
    c = -R.T @ t + delta[:3]
    Rn = so3_exp(delta[3:]) @ R
    return np.concatenate([Rn, (-Rn @ c)[:, None]], axis=1), m, v, delta
