"""Forward-mode dual-number build of the renderer: a second, independent
derivation of the gradient of a rendered image.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): only tests/ use it.

The forward pass of Sec. III-A is written out once more, in plain Python
over a number type that carries, next to each FP64 value, its derivative
with respect to every input at once (a dual number with a vector of
tangents).  Nothing here is shared with gso.c or with the HIP library: the
projection, the EWA covariance (Eq. (1)-(2)), the SH colour, the tile lists
and the compositing (Eq. (3)-(4)) are restated from their definitions, and
the pose enters as the left perturbation T(tau) = Exp(tau) T of Sec. III-B at
tau = 0, whose first-order part is R -> (I + [phi]x) R, t -> (I + [phi]x) t
+ rho.  Discrete decisions (culling, tile rects, depth order, the opacity
clamp, the 1/255 skip, the 1e-4 stop, a colour channel clamped at 0, the
projection-Jacobian clamp) are taken on the values and carry no derivative,
so the tangents are the exact derivatives of the piecewise-smooth render at
the given inputs.  It is meant for scenes of a few Gaussians and images of
a few hundred pixels.
"""
import math

import numpy as np

TILE = 16
NEAR = 0.2
DILATION = 0.3
JCLAMP = 1.3
LAMBDA_FLOOR = 0.1
ALPHA_MAX = 0.99
ALPHA_MIN = 1.0 / 255.0
T_MIN = 1e-4


class Dual:
    """A value and its tangents (numpy vector, one entry per input)."""
    __slots__ = ("v", "d")

    def __init__(self, v, d):
        self.v = float(v)
        self.d = d

    def __add__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v + o.v, self.d + o.d)
        return Dual(self.v + o, self.d)

    __radd__ = __add__

    def __sub__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v - o.v, self.d - o.d)
        return Dual(self.v - o, self.d)

    def __rsub__(self, o):
        return Dual(o - self.v, -self.d)

    def __mul__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v * o.v, self.d * o.v + o.d * self.v)
        return Dual(self.v * o, self.d * o)

    __rmul__ = __mul__

    def __truediv__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v / o.v, (self.d * o.v - o.d * self.v) / (o.v * o.v))
        return Dual(self.v / o, self.d / o)

    def __rtruediv__(self, o):
        return Dual(o / self.v, -o * self.d / (self.v * self.v))

    def __neg__(self):
        return Dual(-self.v, -self.d)


def dsqrt(x):
    r = math.sqrt(x.v)
    return Dual(r, x.d / (2.0 * r))


def dexp(x):
    e = math.exp(x.v)
    return Dual(e, x.d * e)


class _Tangents:
    """Hands out the input variables: each gets a unit tangent of its own."""

    def __init__(self, count):
        self.count = count
        self.next = 0
        self.zero = np.zeros(count)

    def var(self, value):
        d = np.zeros(self.count)
        d[self.next] = 1.0
        self.next += 1
        return Dual(value, d)

    def const(self, value):
        return Dual(value, self.zero)


def _sh_basis(deg, x, y, z):
    """Real SH basis up to degree 3, Condon-Shortley phase, m = -l..l."""
    rpi = math.sqrt(math.pi)
    Y = [Dual(1.0 / (2.0 * rpi), x.d * 0.0)]
    if deg >= 1:
        c = math.sqrt(3.0) / (2.0 * rpi)
        Y += [-c * y, c * z, -c * x]
    if deg >= 2:
        c1 = math.sqrt(15.0) / (2.0 * rpi)
        c2 = math.sqrt(5.0) / (4.0 * rpi)
        c3 = math.sqrt(15.0) / (4.0 * rpi)
        Y += [c1 * (x * y), -c1 * (y * z), c2 * (2.0 * (z * z) - x * x - y * y),
              -c1 * (x * z), c3 * (x * x - y * y)]
    if deg >= 3:
        a = math.sqrt(35.0 / 2.0) / (4.0 * rpi)
        b = math.sqrt(105.0) / (2.0 * rpi)
        c = math.sqrt(21.0 / 2.0) / (4.0 * rpi)
        d = math.sqrt(7.0) / (4.0 * rpi)
        e = math.sqrt(105.0) / (4.0 * rpi)
        r2 = x * x + y * y
        Y += [-a * (y * (3.0 * (x * x) - y * y)),
              b * (x * y * z),
              -c * (y * (4.0 * (z * z) - r2)),
              d * (z * (2.0 * (z * z) - 3.0 * (x * x) - 3.0 * (y * y))),
              -c * (x * (4.0 * (z * z) - r2)),
              e * (z * (x * x - y * y)),
              -a * (x * (x * x - 3.0 * (y * y)))]
    return Y


def render_with_tangents(scene, cam, pose):
    """Renders the scene and returns (values [3, h, w], tangents [3, h, w, K],
    layout) where tangent k is the derivative with respect to input k.
    Inputs are ordered Gaussian by Gaussian (means 3, scales 3, quats 4,
    opacity 1, sh S x 3), then the pose twist tau = (rho, phi); `layout`
    maps each group name to the slice of its entries, as arrays shaped like
    the group."""
    means = np.asarray(scene.means, np.float64)
    scales = np.asarray(scene.scales, np.float64)
    quats = np.asarray(scene.quats, np.float64)
    opac = np.asarray(scene.opacities, np.float64)
    deg = int(scene.sh_degree)
    S = (deg + 1) ** 2
    sh = np.asarray(scene.sh, np.float64).reshape(len(means), S, 3)
    n = len(means)
    per = 11 + 3 * S
    K = n * per + 6
    tg = _Tangents(K)

    pose = np.asarray(pose, np.float64).reshape(3, 4)
    # the twist tau = (rho, phi) takes the last six tangents
    unit = lambda k: np.eye(1, K, k)[0]
    rho_d = [unit(n * per + k) for k in range(3)]
    phi_d = [unit(n * per + 3 + k) for k in range(3)]
    # Exp(tau) T to first order: R' = (I + [phi]x) R, t' = (I + [phi]x) t + rho
    z0 = tg.zero
    px = [[z0, -phi_d[2], phi_d[1]], [phi_d[2], z0, -phi_d[0]], [-phi_d[1], phi_d[0], z0]]
    Rc = [[Dual(pose[r, c], sum(px[r][k] * pose[k, c] for k in range(3))) for c in range(3)]
          for r in range(3)]
    tc = [Dual(pose[r, 3], sum(px[r][k] * pose[k, 3] for k in range(3)) + rho_d[r])
          for r in range(3)]

    W, H = int(cam.width), int(cam.height)
    roi = getattr(cam, "roi", None) or (0, 0, W, H)
    rx0, ry0, rw, rh = (int(x) for x in roi)
    gw, gh = (rw + TILE - 1) // TILE, (rh + TILE - 1) // TILE
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    bg = [float(b) for b in (getattr(cam, "bg", None) or (0.0, 0.0, 0.0))]
    limx = JCLAMP * 0.5 * W / fx
    limy = JCLAMP * 0.5 * H / fy

    # camera centre o_c = -R'^T t'
    oc = [-(Rc[0][k] * tc[0] + Rc[1][k] * tc[1] + Rc[2][k] * tc[2]) for k in range(3)]

    splats = []
    for i in range(n):
        mu = [tg.var(means[i, k]) for k in range(3)]
        s = [tg.var(scales[i, k]) for k in range(3)]
        q = [tg.var(quats[i, k]) for k in range(4)]
        o = tg.var(opac[i])
        f = [[tg.var(sh[i, j, c]) for c in range(3)] for j in range(S)]
        p = [Rc[r][0] * mu[0] + Rc[r][1] * mu[1] + Rc[r][2] * mu[2] + tc[r] for r in range(3)]
        z = p[2]
        if not z.v > NEAR:
            continue
        u = fx * p[0] / z + (cx - 0.5)
        v = fy * p[1] / z + (cy - 0.5)
        xz, yz = p[0] / z, p[1] / z
        if xz.v < -limx or xz.v > limx:
            xz = tg.const(-limx if xz.v < 0 else limx)
        if yz.v < -limy or yz.v > limy:
            yz = tg.const(-limy if yz.v < 0 else limy)
        zero = tg.const(0.0)
        J = [[fx / z, zero, -fx * xz / z], [zero, fy / z, -fy * yz / z]]
        # Eq. (1): unit quaternion -> rotation, Sigma = R diag(s^2) R^T
        nq = dsqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3])
        w, x, y, zz = (c / nq for c in q)
        Rq = [[1.0 - 2.0 * (y * y + zz * zz), 2.0 * (x * y - w * zz), 2.0 * (x * zz + w * y)],
              [2.0 * (x * y + w * zz), 1.0 - 2.0 * (x * x + zz * zz), 2.0 * (y * zz - w * x)],
              [2.0 * (x * zz - w * y), 2.0 * (y * zz + w * x), 1.0 - 2.0 * (x * x + y * y)]]
        s2 = [sk * sk for sk in s]
        Sig = [[sum((Rq[a][k] * s2[k] * Rq[b][k] for k in range(3)), zero) for b in range(3)]
               for a in range(3)]
        # Eq. (2): Sigma_hat = J R' Sigma R'^T J^T + dilation
        JW = [[sum((J[a][k] * Rc[k][b] for k in range(3)), zero) for b in range(3)]
              for a in range(2)]
        M2 = [[sum((JW[a][k] * Sig[k][c] for k in range(3)), zero) for c in range(3)]
              for a in range(2)]
        ca = sum((M2[0][k] * JW[0][k] for k in range(3)), zero) + DILATION
        cb = sum((M2[0][k] * JW[1][k] for k in range(3)), zero)
        cc = sum((M2[1][k] * JW[1][k] for k in range(3)), zero) + DILATION
        det = ca * cc - cb * cb
        if not det.v > 0:
            continue
        A, B, C = cc / det, -cb / det, ca / det
        mid = 0.5 * (ca.v + cc.v)
        lam = mid + math.sqrt(max(LAMBDA_FLOOR, mid * mid - det.v))
        r = int(math.ceil(3.0 * math.sqrt(lam)))
        tx0 = min(max(math.floor((u.v - r) / TILE) - rx0 // TILE, 0), gw)
        ty0 = min(max(math.floor((v.v - r) / TILE) - ry0 // TILE, 0), gh)
        tx1 = min(max(math.floor((u.v + r + TILE - 1) / TILE) - rx0 // TILE, 0), gw)
        ty1 = min(max(math.floor((v.v + r + TILE - 1) / TILE) - ry0 // TILE, 0), gh)
        if tx1 <= tx0 or ty1 <= ty0:
            continue
        # SH colour from the direction (mu - o_c) / |mu - o_c|
        dvec = [mu[k] - oc[k] for k in range(3)]
        dn = dsqrt(dvec[0] * dvec[0] + dvec[1] * dvec[1] + dvec[2] * dvec[2])
        Y = _sh_basis(deg, dvec[0] / dn, dvec[1] / dn, dvec[2] / dn)
        col = []
        for ch in range(3):
            c = sum((f[j][ch] * Y[j] for j in range(S)), zero) + 0.5
            col.append(c if not c.v < 0 else tg.const(0.0))
        splats.append(dict(i=i, u=u, v=v, A=A, B=B, C=C, o=o, col=col,
                           key=float(np.float32(z.v)), rect=(tx0, ty0, tx1, ty1)))
    assert tg.next == n * per, "every Gaussian input handed out"

    val = np.zeros((3, rh, rw))
    tan = np.zeros((3, rh, rw, K))
    for ty in range(gh):
        for tx in range(gw):
            lst = sorted((s for s in splats
                          if s["rect"][0] <= tx < s["rect"][2] and s["rect"][1] <= ty < s["rect"][3]),
                         key=lambda s: (s["key"], s["i"]))
            for yy in range(ty * TILE, min((ty + 1) * TILE, rh)):
                for xx in range(tx * TILE, min((tx + 1) * TILE, rw)):
                    pxf, pyf = float(rx0 + xx), float(ry0 + yy)
                    T = tg.const(1.0)
                    acc = [tg.const(0.0) for _ in range(3)]
                    for s in lst:
                        dx, dy = s["u"] - pxf, s["v"] - pyf
                        power = -0.5 * (s["A"] * dx * dx + s["C"] * dy * dy) - s["B"] * dx * dy
                        if power.v > 0:
                            continue
                        a = s["o"] * dexp(power)
                        if a.v > ALPHA_MAX:
                            a = tg.const(ALPHA_MAX)
                        if a.v < ALPHA_MIN:
                            continue
                        if T.v * (1.0 - a.v) < T_MIN:
                            break
                        w_ = a * T
                        for ch in range(3):
                            acc[ch] = acc[ch] + s["col"][ch] * w_
                        T = T * (1.0 - a)
                    for ch in range(3):
                        out = acc[ch] + T * bg[ch]
                        val[ch, yy, xx] = out.v
                        tan[ch, yy, xx] = out.d
    layout = {}
    base = np.arange(n * per).reshape(n, per)
    off = 0
    for name, width in (("means", 3), ("scales", 3), ("quats", 4), ("opacities", 1), ("sh", 3 * S)):
        sl = base[:, off:off + width]
        layout[name] = sl[:, 0] if name == "opacities" else (sl.reshape(n, S, 3) if name == "sh" else sl)
        off += width
    layout["pose"] = np.arange(n * per, K)
    return val, tan, layout


def gradient_of_linear_loss(scene, cam, pose, weights):
    """(image, gradients) of L = <weights, image> by forward mode: every
    group of the scene and the pose twist (rho, phi), from the tangents."""
    val, tan, layout = render_with_tangents(scene, cam, pose)
    g = np.tensordot(np.asarray(weights, np.float64), tan, axes=3)
    return val, {k: g[idx] for k, idx in layout.items()}
