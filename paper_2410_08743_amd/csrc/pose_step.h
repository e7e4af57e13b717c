// pose_step.h -- the tangent-space Adam step on a pose (Sec. III-B: the
// pose is T = Exp(tau) T0, gradients are taken on the twist tau and the
// update is retracted on the left), shared by the standalone Adam kernel and
// the backward's final pose reduction, which can apply the step itself.
#pragma once

#include "gsp_internal.h"

namespace gsp {

// SE(3) exponential of (rho, phi) in FP64, composed on the left of T.
__device__ inline void se3_retract_left(const double d[6], float *T) {
    const double px = d[3], py = d[4], pz = d[5];
    const double th2 = px * px + py * py + pz * pz, th = sqrt(th2);
    double A, B, C;   // sin t / t, (1 - cos t) / t^2, (t - sin t) / t^3
    if (th < 1e-4) {
        A = 1 - th2 / 6 + th2 * th2 / 120;
        B = 0.5 - th2 / 24 + th2 * th2 / 720;
        C = 1.0 / 6 - th2 / 120 + th2 * th2 / 5040;
    } else {
        A = sin(th) / th;
        B = (1 - cos(th)) / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    const double K[9] = {0, -pz, py, pz, 0, -px, -py, px, 0};
    double K2[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++)
            K2[3 * r + c] = K[3 * r] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
    double E[12];
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++) {
            const double I = r == c ? 1.0 : 0.0;
            E[4 * r + c] = I + A * K[3 * r + c] + B * K2[3 * r + c];
        }
        double tr = 0;
        for (int c = 0; c < 3; c++) {
            const double I = r == c ? 1.0 : 0.0;
            tr += (I + B * K[3 * r + c] + C * K2[3 * r + c]) * d[c];
        }
        E[4 * r + 3] = tr;
    }
    double out[12];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 4; c++) {
            double s = E[4 * r] * T[c] + E[4 * r + 1] * T[4 + c] + E[4 * r + 2] * T[8 + c];
            if (c == 3) s += E[4 * r + 3];
            out[4 * r + c] = s;
        }
    for (int k = 0; k < 12; k++) T[k] = (float)out[k];
}

// SO(3) exponential of phi composed on the left of the rotation of T, with
// the camera centre c kept: T = [R | -R c] -> [Exp(phi) R | -Exp(phi) R c'],
// c' = c + dc (the T x SO(3) step).
__device__ inline void tso3_step(const double dc[3], const double phi[3], float *T) {
    const double px = phi[0], py = phi[1], pz = phi[2];
    const double th2 = px * px + py * py + pz * pz, th = sqrt(th2);
    double A, B;   // sin t / t, (1 - cos t) / t^2
    if (th < 1e-4) {
        A = 1 - th2 / 6 + th2 * th2 / 120;
        B = 0.5 - th2 / 24 + th2 * th2 / 720;
    } else {
        A = sin(th) / th;
        B = (1 - cos(th)) / th2;
    }
    const double K[9] = {0, -pz, py, pz, 0, -px, -py, px, 0};
    double E[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            const double k2 = K[3 * r] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
            E[3 * r + c] = (r == c ? 1.0 : 0.0) + A * K[3 * r + c] + B * k2;
        }
    double R[9], t[3];
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++) R[3 * r + c] = T[4 * r + c];
        t[r] = T[4 * r + 3];
    }
    double cc[3];
    for (int k = 0; k < 3; k++) cc[k] = -(R[k] * t[0] + R[3 + k] * t[1] + R[6 + k] * t[2]) + dc[k];
    double Rn[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++)
            Rn[3 * r + c] = E[3 * r] * R[c] + E[3 * r + 1] * R[3 + c] + E[3 * r + 2] * R[6 + c];
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++) T[4 * r + c] = (float)Rn[3 * r + c];
        T[4 * r + 3] = (float)(-(Rn[3 * r] * cc[0] + Rn[3 * r + 1] * cc[1] + Rn[3 * r + 2] * cc[2]));
    }
}

// One Adam step of view i from its loaded state: k is the step's count
// (steps[i] + 1), gv the pose gradient, m0 / v0 the moments and T0 the pose
// (updated in place, then stored); writes steps[i], m, v and poses.
__device__ inline void pose_adam_apply(int i, int k, double gv[6], const double m0[6],
                                       const double v0[6], float T0[12], float *poses, float *m,
                                       float *v, int32_t *steps, const gsp_adam_params &p) {
    steps[i] = k;
    double lr = p.lr_start;
    if (p.total_steps > 1) {
        const double frac = fmin((double)(k - 1), (double)(p.total_steps - 1)) / (p.total_steps - 1);
        lr = p.lr_end + 0.5 * ((double)p.lr_start - p.lr_end) * (1.0 + cos(M_PI * frac));
    }
    const double b1 = p.beta1, b2 = p.beta2;
    const double c1 = 1.0 - pow(b1, (double)k), c2 = 1.0 - pow(b2, (double)k);
    const bool tso3 = p.parametrization == GSP_POSE_T_SO3;
    if (tso3) {   // dL/dc = -R^T dL/drho; the rotation part is unchanged
        const float *T = T0;
        double gc[3];
        for (int k2 = 0; k2 < 3; k2++)
            gc[k2] = -((double)T[k2] * gv[0] + (double)T[4 + k2] * gv[1] + (double)T[8 + k2] * gv[2]);
        for (int k2 = 0; k2 < 3; k2++) gv[k2] = gc[k2];
    }
    double delta[6];
    for (int e = 0; e < 6; e++) {
        const double g = gv[e];
        const double mm = b1 * m0[e] + (1.0 - b1) * g;
        const double vv = b2 * v0[e] + (1.0 - b2) * g * g;
        m[6 * i + e] = (float)mm;
        v[6 * i + e] = (float)vv;
        delta[e] = -lr * (mm / c1) / (sqrt(vv / c2) + (double)p.eps);
    }
    if (tso3)
        tso3_step(delta, delta + 3, T0);
    else
        se3_retract_left(delta, T0);
#pragma unroll
    for (int e = 0; e < 12; e++) poses[12 * i + e] = T0[e];
}

}  // namespace gsp
