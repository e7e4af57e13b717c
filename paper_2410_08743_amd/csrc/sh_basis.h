// sh_basis.h -- real spherical harmonics up to degree 3 at a direction
// (Sec. III-A: the colour of a splat is SH(f, d)).  Condon-Shortley phase,
// ordered m = -l..l within each degree.  The constants are the
// normalisations sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (times sqrt 2 for
// m != 0) folded with the polynomial coefficients of each basis function.
#pragma once

#include <hip/hip_runtime.h>

namespace gsp {

namespace shc {
constexpr double c0 = 0.28209479177387814;   // 1 / (2 sqrt(pi))
constexpr double c1 = 0.4886025119029199;    // sqrt(3) / (2 sqrt(pi))
constexpr double c2a = 1.0925484305920792;   // sqrt(15) / (2 sqrt(pi))
constexpr double c2b = 0.31539156525252005;  // sqrt(5) / (4 sqrt(pi))
constexpr double c2c = 0.5462742152960396;   // sqrt(15) / (4 sqrt(pi))
constexpr double c3a = 0.5900435899266435;   // sqrt(35/2) / (4 sqrt(pi))
constexpr double c3b = 2.890611442640554;    // sqrt(105) / (2 sqrt(pi))
constexpr double c3c = 0.4570457994644658;   // sqrt(21/2) / (4 sqrt(pi))
constexpr double c3d = 0.3731763325901154;   // sqrt(7) / (4 sqrt(pi))
constexpr double c3e = 1.445305721320277;    // sqrt(105) / (4 sqrt(pi))
}  // namespace shc

// Y[k] for k < (D+1)^2 at unit direction (x, y, z).
template <int D, typename T>
__device__ __forceinline__ void sh_eval(T x, T y, T z, T *Y) {
    Y[0] = T(shc::c0);
    if constexpr (D >= 1) {
        Y[1] = -T(shc::c1) * y;
        Y[2] = T(shc::c1) * z;
        Y[3] = -T(shc::c1) * x;
    }
    if constexpr (D >= 2) {
        const T xx = x * x, yy = y * y, zz = z * z;
        Y[4] = T(shc::c2a) * x * y;
        Y[5] = -T(shc::c2a) * y * z;
        Y[6] = T(shc::c2b) * (T(2) * zz - xx - yy);
        Y[7] = -T(shc::c2a) * x * z;
        Y[8] = T(shc::c2c) * (xx - yy);
        if constexpr (D >= 3) {
            Y[9] = -T(shc::c3a) * y * (T(3) * xx - yy);
            Y[10] = T(shc::c3b) * x * y * z;
            Y[11] = -T(shc::c3c) * y * (T(4) * zz - xx - yy);
            Y[12] = T(shc::c3d) * z * (T(2) * zz - T(3) * xx - T(3) * yy);
            Y[13] = -T(shc::c3c) * x * (T(4) * zz - xx - yy);
            Y[14] = T(shc::c3e) * z * (xx - yy);
            Y[15] = -T(shc::c3a) * x * (xx - T(3) * yy);
        }
    }
}

// Gradient of sum_k w[k] Y_k(x, y, z) with respect to (x, y, z), each Y_k
// differentiated as a polynomial (the caller projects out the radial part).
template <int D, typename T>
__device__ __forceinline__ void sh_weighted_grad(T x, T y, T z, const T *w, T g[3]) {
    g[0] = g[1] = g[2] = T(0);
    if constexpr (D >= 1) {
        g[1] -= T(shc::c1) * w[1];
        g[2] += T(shc::c1) * w[2];
        g[0] -= T(shc::c1) * w[3];
    }
    if constexpr (D >= 2) {
        const T a = T(shc::c2a), b = T(shc::c2b), c = T(shc::c2c);
        g[0] += a * y * w[4];
        g[1] += a * x * w[4];
        g[1] -= a * z * w[5];
        g[2] -= a * y * w[5];
        g[0] -= T(2) * b * x * w[6];
        g[1] -= T(2) * b * y * w[6];
        g[2] += T(4) * b * z * w[6];
        g[0] -= a * z * w[7];
        g[2] -= a * x * w[7];
        g[0] += T(2) * c * x * w[8];
        g[1] -= T(2) * c * y * w[8];
    }
    if constexpr (D >= 3) {
        const T xx = x * x, yy = y * y, zz = z * z;
        const T a = T(shc::c3a), b = T(shc::c3b), c = T(shc::c3c), d = T(shc::c3d),
                e = T(shc::c3e);
        // Y9 = -a (3 x^2 y - y^3)
        g[0] += -T(6) * a * x * y * w[9];
        g[1] += -a * (T(3) * xx - T(3) * yy) * w[9];
        // Y10 = b x y z
        g[0] += b * y * z * w[10];
        g[1] += b * x * z * w[10];
        g[2] += b * x * y * w[10];
        // Y11 = -c (4 y z^2 - x^2 y - y^3)
        g[0] += T(2) * c * x * y * w[11];
        g[1] += -c * (T(4) * zz - xx - T(3) * yy) * w[11];
        g[2] += -T(8) * c * y * z * w[11];
        // Y12 = d (2 z^3 - 3 x^2 z - 3 y^2 z)
        g[0] += -T(6) * d * x * z * w[12];
        g[1] += -T(6) * d * y * z * w[12];
        g[2] += d * (T(6) * zz - T(3) * xx - T(3) * yy) * w[12];
        // Y13 = -c (4 x z^2 - x^3 - x y^2)
        g[0] += -c * (T(4) * zz - T(3) * xx - yy) * w[13];
        g[1] += T(2) * c * x * y * w[13];
        g[2] += -T(8) * c * x * z * w[13];
        // Y14 = e (x^2 z - y^2 z)
        g[0] += T(2) * e * x * z * w[14];
        g[1] += -T(2) * e * y * z * w[14];
        g[2] += e * (xx - yy) * w[14];
        // Y15 = -a (x^3 - 3 x y^2)
        g[0] += -a * (T(3) * xx - T(3) * yy) * w[15];
        g[1] += T(6) * a * x * y * w[15];
    }
}

}  // namespace gsp
