// preprocess_bwd.hip -- chain rule from the per-splat 2D gradients to the
// Gaussian parameters and to each view's se(3) pose twist.
//
// Sec. III-B, Eq. (7): the pose gradient collects, over Gaussians, the 2D
// mean term (through mu^c = T mu, Eq. (8)/(10): d mu^c / d tau = (I | -[mu^c]x)),
// the 2D covariance term (through J(mu^c) and through R_c, Eq. (12)-(13):
// dR_c / d phi_k = [e_k]x R_c) and the colour term (through the camera
// centre o_c = -R_c^T t_c, which moves by -R_c^T rho under the left
// perturbation).  Per Gaussian, with g = dL/dmu^c, G_W = dL/dR_c (from
// Sigma_hat = J R_c Sigma R_c^T J^T) and h = dL/do_c:
//   dL/drho += g - R_c h,   dL/dphi += mu^c x g + vee(G_W R_c^T).
//
// MI355X design: a first kernel walks the instance slots in their emission
// order (visible splats in index order, each splat's slots contiguous), in
// windows of balanced size, and sums each splat's slots in a fixed order
// into its 2D gradient.  The chain-rule kernel then runs one thread per
// Gaussian over the call's views, geometry in FP64 (the FP64 vector rate
// equals unpacked FP32), SH in FP32.  Gaussian gradients are summed over
// views in registers and written once; the six pose sums per view are
// reduced with wavefront shuffles into per-wavefront partials (no barrier
// inside the loop over views), and one block per view adds the partials in
// a fixed order.  No atomics anywhere, so the result is bit-reproducible and
// a view's pose gradient does not depend on which other views share the
// launch.
#include <cstring>

#include "block_ops.h"
#include "gsp_internal.h"
#include "pose_step.h"
#include "sh_basis.h"

namespace gsp {

struct PbArgs {
    GaussiansK g;
    const float *poses;
    const uint32_t *tiles;
    const uint32_t *counters;
    const float *slots;     // [cap][9]
    float *grad2d;          // [vn][9]
    double *posepart;       // [V][nblk * kPoseRowsPerBlock][6]: one row per wavefront
    gsp_grads out;
    size_t cap, vn;
    int nblk;
    bool accumulate;
};

// d R(qhat) / d qhat . G for a unit quaternion (w, x, y, z).
__device__ __forceinline__ void rot_vjp(double w, double x, double y, double z, const double Gm[9],
                                        double out[4]) {
    out[0] = 2 * (-z * Gm[1] + y * Gm[2] + z * Gm[3] - x * Gm[5] - y * Gm[6] + x * Gm[7]);
    out[1] = 2 * (y * Gm[1] + z * Gm[2] + y * Gm[3] - 2 * x * Gm[4] - w * Gm[5] + z * Gm[6] +
                  w * Gm[7] - 2 * x * Gm[8]);
    out[2] = 2 * (-2 * y * Gm[0] + x * Gm[1] + w * Gm[2] + x * Gm[3] + z * Gm[5] - w * Gm[6] +
                  z * Gm[7] - 2 * y * Gm[8]);
    out[3] = 2 * (-2 * z * Gm[0] - w * Gm[1] + x * Gm[2] + w * Gm[3] - 2 * z * Gm[4] + y * Gm[5] +
                  x * Gm[6] + y * Gm[7]);
}

// 2D gradient of each splat: the sum of its instance slots in slot order (one
// running sum from zero, first instance to last, and within an instance its
// rasterizer parts in order).  One block per work window: the
// window's slots form one contiguous range, which the block copies into LDS
// with all of each thread's loads in flight at once; the (splat, component)
// pairs are then spread over the threads, nine neighbouring threads per
// splat.  Slots past the first kWindow of the range -- the tail of a long last
// splat -- are read from global memory.  A slot the backward rasterizer did
// not write (flag 0: no pixel of that strip blended the entry) counts as zero.
constexpr int kSlotFloats = 9 * kSplitBwd;   // one 9-float slot per backward part
constexpr int kSlotPerThread = kWindow * kSlotFloats / kWindowThreads;

__global__ __launch_bounds__(kWindowThreads) void k_slot_reduce(const uint32_t *offk,
                                                                const uint2 *wstart,
                                                                const uint32_t *counters,
                                                                const float *slots,
                                                                const uint8_t *flags,
                                                                float *grad2d, int vn) {
    __shared__ float s_sl[kWindow * kSlotFloats];
    __shared__ uint8_t s_fl[kWindow * kSplitBwd];
    __shared__ uint32_t s_off[kWindow + 1];
    const int b = blockIdx.x;
    if (counters[kCntOverflow] != 0u) {
        // no instance was emitted: every 2D gradient is zero
        for (size_t f = (size_t)b * kWindowThreads + threadIdx.x; f < 9 * (size_t)vn;
             f += (size_t)gridDim.x * kWindowThreads)
            grad2d[f] = 0.f;
        return;
    }
    if ((uint32_t)b >= counters[kCntWin]) return;
    // the window's first splat and first slot, and the next window's
    const uint2 w0 = wstart[b], w1 = wstart[b + 1];
    const uint32_t kb = w0.x, ke = w1.x;
    const int nk = (int)(ke - kb);   // at most kWindow
    const uint32_t e0 = w0.y, ne = w1.y - e0;
    const uint32_t nf = (uint32_t)kSlotFloats * min(ne, (uint32_t)kWindow);
    const float *src = slots + kSlotFloats * (size_t)e0;
    const uint8_t *fsrc = flags + kSplitBwd * (size_t)e0;
    const uint32_t nfl = (uint32_t)kSplitBwd * min(ne, (uint32_t)kWindow);
    for (uint32_t f = threadIdx.x; f < nfl; f += kWindowThreads) s_fl[f] = fsrc[f];
    float tmp[kSlotPerThread];
#pragma unroll
    for (int r = 0; r < kSlotPerThread; r++) {
        const uint32_t f = (uint32_t)(r * kWindowThreads + threadIdx.x);
        tmp[r] = f < nf ? src[f] : 0.f;
    }
    for (int j = threadIdx.x; j < nk; j += kWindowThreads) s_off[j] = offk[kb + j] - e0;
    if (threadIdx.x == 0) s_off[nk] = ne;
#pragma unroll
    for (int r = 0; r < kSlotPerThread; r++) s_sl[r * kWindowThreads + threadIdx.x] = tmp[r];
    __syncthreads();
    for (int item = threadIdx.x; item < 9 * nk; item += kWindowThreads) {
        const int j = item / 9, c = item - 9 * j;
        const uint32_t lo = s_off[j], hi = s_off[j + 1];
        const uint32_t mid = min(hi, (uint32_t)kWindow);
        float d = 0.f;
        uint32_t e = lo;
        // slots in LDS, kLdsBatch reads in flight, added in slot order
        constexpr int kLdsBatch = 4;
        for (; e + kLdsBatch <= mid; e += kLdsBatch) {
            float v[kLdsBatch][kSplitBwd];
            bool fl[kLdsBatch][kSplitBwd];
#pragma unroll
            for (int u = 0; u < kLdsBatch; u++)
#pragma unroll
                for (int p = 0; p < kSplitBwd; p++) {
                    v[u][p] = s_sl[kSlotFloats * (e + u) + 9 * p + c];
                    fl[u][p] = s_fl[kSplitBwd * (e + u) + p] != 0;
                }
#pragma unroll
            for (int u = 0; u < kLdsBatch; u++)
#pragma unroll
                for (int p = 0; p < kSplitBwd; p++) d += fl[u][p] ? v[u][p] : 0.f;
        }
        for (; e < mid; e++) {
#pragma unroll
            for (int p = 0; p < kSplitBwd; p++) {
                const float v = s_sl[kSlotFloats * e + 9 * p + c];
                d += s_fl[kSplitBwd * e + p] ? v : 0.f;
            }
        }
        // the tail past the window, from global memory: the loads of
        // kTailBatch slots are issued together, then added in slot order
        constexpr int kTailBatch = 8;
        for (; e + kTailBatch <= hi; e += kTailBatch) {
            float v[kTailBatch][kSplitBwd];
            uint8_t fl[kTailBatch][kSplitBwd];
#pragma unroll
            for (int u = 0; u < kTailBatch; u++)
#pragma unroll
                for (int p = 0; p < kSplitBwd; p++) {
                    v[u][p] = src[kSlotFloats * (size_t)(e + u) + 9 * p + c];
                    fl[u][p] = fsrc[kSplitBwd * (size_t)(e + u) + p];
                }
#pragma unroll
            for (int u = 0; u < kTailBatch; u++)
#pragma unroll
                for (int p = 0; p < kSplitBwd; p++) d += fl[u][p] ? v[u][p] : 0.f;
        }
        for (; e < hi; e++) {
#pragma unroll
            for (int p = 0; p < kSplitBwd; p++) {
                const float v = src[kSlotFloats * (size_t)e + 9 * p + c];
                d += fsrc[kSplitBwd * (size_t)e + p] ? v : 0.f;
            }
        }
        grad2d[9 * ((size_t)kb + j) + c] = d;
    }
}

// Symmetric 3 x 3 matrices are kept as their six upper entries
// (xx, xy, xz, yy, yz, zz).
__host__ __device__ constexpr int sym3(int r, int c) {
    return r <= c ? (r == 0 ? c : (r == 1 ? 2 + c : 5)) : (c == 0 ? r : (c == 1 ? 2 + r : 5));
}

// Rotation of the unit quaternion q / |q|, with |q| returned.
__device__ __forceinline__ double quat_rot(const float *qp, double qh[4], double Rq[9]) {
    double q[4];
#pragma unroll
    for (int k = 0; k < 4; k++) q[k] = qp[k];
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
#pragma unroll
    for (int k = 0; k < 4; k++) qh[k] = q[k] / qn;
    const double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
    Rq[0] = 1 - 2 * (y * y + z * z); Rq[1] = 2 * (x * y - w * z); Rq[2] = 2 * (x * z + w * y);
    Rq[3] = 2 * (x * y + w * z); Rq[4] = 1 - 2 * (x * x + z * z); Rq[5] = 2 * (y * z - w * x);
    Rq[6] = 2 * (x * z - w * y); Rq[7] = 2 * (y * z + w * x); Rq[8] = 1 - 2 * (x * x + y * y);
    return qn;
}

// Resident waves per SIMD.  What crosses the loop over views stays in
// registers (the SH coefficients, the mean, the six entries of Sigma and the
// gradient sums); the rotation and scales are read again at the end.  At SH
// degree 3 both variants take two waves: 213 registers for the pose-only
// kernel, 254 with every Gaussian gradient.  (Reading the pose-only
// kernel's SH coefficients with each view's inputs instead fits three
// waves, 160 registers, and measured no faster.)
#ifndef GSP_PB_WAVES_POSE
#define GSP_PB_WAVES_POSE 2
#endif
#ifndef GSP_PB_WAVES_GAUSS
#define GSP_PB_WAVES_GAUSS 2
#endif
template <bool WANT_GAUSS>
constexpr int pb_waves() { return WANT_GAUSS ? GSP_PB_WAVES_GAUSS : GSP_PB_WAVES_POSE; }

template <int D, bool WANT_GAUSS>
__global__ __launch_bounds__(kPoseReduceBlock) __attribute__((amdgpu_waves_per_eu(pb_waves<WANT_GAUSS>()))) void k_preprocess_bwd(PbArgs a, ViewsK views) {
    constexpr int S = (D + 1) * (D + 1);
    static_assert(kPoseRowsPerBlock * kWave == kPoseReduceBlock, "one pose row per wavefront");
    const int n = a.g.n;
    const int i = blockIdx.x * kPoseReduceBlock + threadIdx.x;
    const bool valid = i < n;
    const bool ovf = a.counters[kCntOverflow] != 0u;

    double mu[3] = {0, 0, 0};
    double Sig[6] = {0, 0, 0, 0, 0, 0};
    float sh[S * 3];
#pragma unroll
    for (int k = 0; k < S * 3; k++) sh[k] = 0.f;
    if (valid) {
        const float *f = a.g.sh + (size_t)i * (S * 3);
#pragma unroll
        for (int k = 0; k < S * 3; k++) sh[k] = f[k];
#pragma unroll
        for (int k = 0; k < 3; k++) mu[k] = a.g.means[3 * i + k];
        double qh[4], Rq[9], s2[3];
        quat_rot(a.g.quats + 4 * (size_t)i, qh, Rq);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const double s = a.g.scales[3 * i + k];
            s2[k] = s * s;
        }
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
            for (int c = r; c < 3; c++)
                Sig[sym3(r, c)] = Rq[3 * r] * Rq[3 * c] * s2[0] + Rq[3 * r + 1] * Rq[3 * c + 1] * s2[1] +
                                  Rq[3 * r + 2] * Rq[3 * c + 2] * s2[2];
    }

    // gradients summed over views
    double gmu[3] = {0, 0, 0}, gSig[6] = {0, 0, 0, 0, 0, 0}, gop = 0;
    // SH gradient accumulators in LDS ([coefficient][thread], conflict-free),
    // not registers
    __shared__ float s_gsh[WANT_GAUSS ? S * 3 : 1][kPoseReduceBlock];
    if constexpr (WANT_GAUSS) {
#pragma unroll
        for (int k = 0; k < S * 3; k++) s_gsh[k][threadIdx.x] = 0.f;
    }

    for (int v = 0; v < views.count; v++) {
        const ViewK &vw = views.v[v];
        const float *P = a.poses + 12 * v;
        const size_t idx = (size_t)v * n + i;
        double pose6[6] = {0, 0, 0, 0, 0, 0};
        const uint32_t cnt = (valid && !ovf) ? a.tiles[idx] : 0u;
        if (cnt > 0) {
            float d2f[9];
#pragma unroll
            for (int c = 0; c < 9; c++) d2f[c] = a.grad2d[9 * (size_t)idx + c];
            double R[9], t[3];
#pragma unroll
            for (int r = 0; r < 3; r++) {
                R[3 * r] = P[4 * r];
                R[3 * r + 1] = P[4 * r + 1];
                R[3 * r + 2] = P[4 * r + 2];
                t[r] = P[4 * r + 3];
            }
            // colour: viewing direction from the camera centre
            const double ocx = -(R[0] * t[0] + R[3] * t[1] + R[6] * t[2]);
            const double ocy = -(R[1] * t[0] + R[4] * t[1] + R[7] * t[2]);
            const double ocz = -(R[2] * t[0] + R[5] * t[1] + R[8] * t[2]);
            const double wx = mu[0] - ocx, wy = mu[1] - ocy, wz = mu[2] - ocz;
            const double dist = sqrt(wx * wx + wy * wy + wz * wz), idist = 1.0 / dist;
            const double dxn = wx * idist, dyn = wy * idist, dzn = wz * idist;
            const float fxn = (float)dxn, fyn = (float)dyn, fzn = (float)dzn;
            float Y[S];
            sh_eval<D, float>(fxn, fyn, fzn, Y);
            float wgt[S];
#pragma unroll
            for (int k = 0; k < S; k++) wgt[k] = 0.f;
#pragma unroll
            for (int ch = 0; ch < 3; ch++) {
                float shc[S];
#pragma unroll
                for (int k = 0; k < S; k++) shc[k] = sh[3 * k + ch];
                float col = 0.5f;
#pragma unroll
                for (int k = 0; k < S; k++) col = fmaf(shc[k], Y[k], col);
                if (col < 0.f) continue;   // clamped channel: no gradient
                const float gc = d2f[6 + ch];
#pragma unroll
                for (int k = 0; k < S; k++) {
                    wgt[k] = fmaf(gc, shc[k], wgt[k]);
                    if constexpr (WANT_GAUSS)
                        s_gsh[3 * k + ch][threadIdx.x] = fmaf(gc, Y[k], s_gsh[3 * k + ch][threadIdx.x]);
                }
            }
            float gdf[3];
            sh_weighted_grad<D, float>(fxn, fyn, fzn, wgt, gdf);
            const double gd[3] = {gdf[0], gdf[1], gdf[2]};
            const double proj = gd[0] * dxn + gd[1] * dyn + gd[2] * dzn;
            const double gw[3] = {(gd[0] - dxn * proj) * idist, (gd[1] - dyn * proj) * idist,
                                  (gd[2] - dzn * proj) * idist};
#pragma unroll
            for (int k = 0; k < 3; k++) gmu[k] += gw[k];
            // pose twist, translation part through the camera centre:
            // h = dL/do_c = -gw
#pragma unroll
            for (int r = 0; r < 3; r++) pose6[r] = R[3 * r] * gw[0] + R[3 * r + 1] * gw[1] + R[3 * r + 2] * gw[2];
            double p[3];
#pragma unroll
            for (int r = 0; r < 3; r++)
                p[r] = fma(R[3 * r + 2], mu[2], fma(R[3 * r + 1], mu[1], fma(R[3 * r], mu[0], t[r])));
            const double z = p[2], iz = 1.0 / z, iz2 = iz * iz;
            const double fx = vw.fx, fy = vw.fy;
            const double limx = kJClamp * 0.5 * vw.W / fx, limy = kJClamp * 0.5 * vw.H / fy;
            const double xzr = p[0] * iz, yzr = p[1] * iz;
            const bool clx = xzr < -limx || xzr > limx, cly = yzr < -limy || yzr > limy;
            const double xz = fmin(fmax(xzr, -limx), limx), yz = fmin(fmax(yzr, -limy), limy);
            const double j00 = fx * iz, j02 = -fx * xz * iz, j11 = fy * iz, j12 = -fy * yz * iz;
            // rows of T2 = J R_c
            const double ta[3] = {j00 * R[0] + j02 * R[6], j00 * R[1] + j02 * R[7],
                                  j00 * R[2] + j02 * R[8]};
            const double tb[3] = {j11 * R[3] + j12 * R[6], j11 * R[4] + j12 * R[7],
                                  j11 * R[5] + j12 * R[8]};
            double sa[3], sb[3];
#pragma unroll
            for (int r = 0; r < 3; r++) {
                sa[r] = Sig[sym3(r, 0)] * ta[0] + Sig[sym3(r, 1)] * ta[1] + Sig[sym3(r, 2)] * ta[2];
                sb[r] = Sig[sym3(r, 0)] * tb[0] + Sig[sym3(r, 1)] * tb[1] + Sig[sym3(r, 2)] * tb[2];
            }
            const double ca = ta[0] * sa[0] + ta[1] * sa[1] + ta[2] * sa[2] + kDilation;
            const double cb = ta[0] * sb[0] + ta[1] * sb[1] + ta[2] * sb[2];
            const double cc = tb[0] * sb[0] + tb[1] * sb[1] + tb[2] * sb[2] + kDilation;
            const double det = ca * cc - cb * cb, idet2 = 1.0 / (det * det);
            const double dA = d2f[2], dB = d2f[3], dC = d2f[4];
            // conic = inverse of the 2D covariance
            const double dca = (-cc * cc * dA + cb * cc * dB - cb * cb * dC) * idet2;
            const double dcb = (2 * cb * cc * dA - (ca * cc + cb * cb) * dB + 2 * ca * cb * dC) * idet2;
            const double dcc = (-cb * cb * dA + ca * cb * dB - ca * ca * dC) * idet2;
            // dL/dT2 rows: 2 [[dca, dcb/2], [dcb/2, dcc]] T2 Sigma
            double ga[3], gb[3];
#pragma unroll
            for (int r = 0; r < 3; r++) {
                ga[r] = 2 * dca * sa[r] + dcb * sb[r];
                gb[r] = dcb * sa[r] + 2 * dcc * sb[r];
            }
            // dL/dJ = dL/dT2 R_c^T (only the four entries J depends on)
            const double gj00 = ga[0] * R[0] + ga[1] * R[1] + ga[2] * R[2];
            const double gj02 = ga[0] * R[6] + ga[1] * R[7] + ga[2] * R[8];
            const double gj11 = gb[0] * R[3] + gb[1] * R[4] + gb[2] * R[5];
            const double gj12 = gb[0] * R[6] + gb[1] * R[7] + gb[2] * R[8];
            // J and the projected centre -> camera-frame mean
            double gp[3];
            gp[0] = d2f[0] * fx * iz;
            gp[1] = d2f[1] * fy * iz;
            gp[2] = -(d2f[0] * fx * p[0] + d2f[1] * fy * p[1]) * iz2 - (gj00 * fx + gj11 * fy) * iz2;
            if (clx) {
                gp[2] += gj02 * fx * xz * iz2;
            } else {
                gp[0] -= gj02 * fx * iz2;
                gp[2] += gj02 * 2 * fx * p[0] * iz2 * iz;
            }
            if (cly) {
                gp[2] += gj12 * fy * yz * iz2;
            } else {
                gp[1] -= gj12 * fy * iz2;
                gp[2] += gj12 * 2 * fy * p[1] * iz2 * iz;
            }
            // mean (geometry part): R_c^T gp
#pragma unroll
            for (int k = 0; k < 3; k++) gmu[k] += R[k] * gp[0] + R[3 + k] * gp[1] + R[6 + k] * gp[2];
#pragma unroll
            for (int r = 0; r < 3; r++) pose6[r] += gp[r];
            if constexpr (WANT_GAUSS) {
                // dL/dSigma = T2^T Gh T2 (symmetric)
#pragma unroll
                for (int r = 0; r < 3; r++)
#pragma unroll
                    for (int c = r; c < 3; c++)
                        gSig[sym3(r, c)] += dca * ta[r] * ta[c] + 0.5 * dcb * (ta[r] * tb[c] + tb[r] * ta[c]) +
                                            dcc * tb[r] * tb[c];
                gop += d2f[5];
            }
            // dL/dR_c = J^T dL/dT2 =: G_W; the phi part is vee(G_W R_c^T),
            // of which only the antisymmetric entries are needed
            double GW[9];
#pragma unroll
            for (int c = 0; c < 3; c++) {
                GW[c] = j00 * ga[c];
                GW[3 + c] = j11 * gb[c];
                GW[6 + c] = j02 * ga[c] + j12 * gb[c];
            }
            auto bm = [&](int r, int c) {
                return GW[3 * r] * R[3 * c] + GW[3 * r + 1] * R[3 * c + 1] + GW[3 * r + 2] * R[3 * c + 2];
            };
            pose6[3] = p[1] * gp[2] - p[2] * gp[1] + bm(2, 1) - bm(1, 2);
            pose6[4] = p[2] * gp[0] - p[0] * gp[2] + bm(0, 2) - bm(2, 0);
            pose6[5] = p[0] * gp[1] - p[1] * gp[0] + bm(1, 0) - bm(0, 1);
        }
        // per-wavefront sums: no barrier inside the loop over views
        double *const prow =
            a.posepart + ((size_t)v * a.nblk + blockIdx.x) * (kPoseRowsPerBlock * 6) + (threadIdx.x / kWave) * 6;
#pragma unroll
        for (int c = 0; c < 6; c++) {
            const double s = wave_sum(pose6[c]);
            if (threadIdx.x % kWave == 0) prow[c] = s;
        }
    }

    if constexpr (WANT_GAUSS) {
        const gsp_grads &o = a.out;
        const bool acc = a.accumulate;
        if (o.sh) {
            // the block's SH gradients are one contiguous range: coalesced
            __syncthreads();
            const int i0 = blockIdx.x * kPoseReduceBlock;
            const int cnt = min(kPoseReduceBlock, n - i0) * (S * 3);
            float *dst = o.sh + (size_t)i0 * (S * 3);
            for (int e = threadIdx.x; e < cnt; e += kPoseReduceBlock) {
                const float gv = s_gsh[e % (S * 3)][e / (S * 3)];
                dst[e] = (acc ? dst[e] : 0.f) + gv;
            }
        }
        if (!valid) return;
        if (o.means) {
#pragma unroll
            for (int k = 0; k < 3; k++) o.means[3 * i + k] = (acc ? o.means[3 * i + k] : 0.f) + (float)gmu[k];
        }
        if (o.opacities) o.opacities[i] = (acc ? o.opacities[i] : 0.f) + (float)gop;
        if (o.scales || o.quats) {
            double qh[4], Rq[9], sc[3];
            const double qn = quat_rot(a.g.quats + 4 * (size_t)i, qh, Rq);
#pragma unroll
            for (int k = 0; k < 3; k++) sc[k] = a.g.scales[3 * i + k];
            // Sigma = M M^T with M = R_q diag(s): dL/dM = 2 dL/dSigma M (dL/dSigma symmetric)
            double GM[9];
#pragma unroll
            for (int r = 0; r < 3; r++)
#pragma unroll
                for (int c = 0; c < 3; c++)
                    GM[3 * r + c] = 2 * (gSig[sym3(r, 0)] * Rq[c] + gSig[sym3(r, 1)] * Rq[3 + c] +
                                         gSig[sym3(r, 2)] * Rq[6 + c]) * sc[c];
            if (o.scales) {
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const double ds = GM[c] * Rq[c] + GM[3 + c] * Rq[3 + c] + GM[6 + c] * Rq[6 + c];
                    o.scales[3 * i + c] = (acc ? o.scales[3 * i + c] : 0.f) + (float)ds;
                }
            }
            if (o.quats) {
                double GR[9];
#pragma unroll
                for (int r = 0; r < 3; r++)
#pragma unroll
                    for (int c = 0; c < 3; c++) GR[3 * r + c] = GM[3 * r + c] * sc[c];
                double dqh[4];
                rot_vjp(qh[0], qh[1], qh[2], qh[3], GR, dqh);
                const double pr = dqh[0] * qh[0] + dqh[1] * qh[1] + dqh[2] * qh[2] + dqh[3] * qh[3];
#pragma unroll
                for (int k = 0; k < 4; k++)
                    o.quats[4 * i + k] = (acc ? o.quats[4 * i + k] : 0.f) + (float)((dqh[k] - qh[k] * pr) / qn);
            }
        }
    }
}

// dL/dtau of each view: the sum of the chain-rule kernel's per-wavefront
// FP64 partials in a fixed order.  One 256-thread block per view; each
// thread issues all loads of its rows before the first add (one round of
// memory latency per kPoseFinalThreads x kPoseFinalPer rows).
constexpr int kPoseFinalThreads = 256;
constexpr int kPoseFinalPer = 16;   // partial rows per thread held in flight

__global__ __launch_bounds__(kPoseFinalThreads) void k_pose_final(const double *posepart, int nrows,
                                                                  float *dpose, bool accumulate,
                                                                  PoseAdamK ad, bool adam) {
    __shared__ double red[6][kPoseFinalThreads];
    __shared__ float dp6[6];
    const int v = blockIdx.x, t = threadIdx.x;
    // with the Adam step: its state, read before the rows (one round of
    // memory latency for both)
    uint32_t ovf = 0u;
    int k = 0;
    double m0[6] = {0, 0, 0, 0, 0, 0}, v0[6] = {0, 0, 0, 0, 0, 0};
    float T0[12];
#pragma unroll
    for (int e = 0; e < 12; e++) T0[e] = 0.f;
    if (adam && t == 0) {
        ovf = ad.guard[kCntOverflow];
        k = ad.steps[v] + 1;
#pragma unroll
        for (int e = 0; e < 6; e++) {
            m0[e] = ad.m[6 * v + e];
            v0[e] = ad.v[6 * v + e];
        }
#pragma unroll
        for (int e = 0; e < 12; e++) T0[e] = ad.poses[12 * v + e];
    }
    const double *src = posepart + (size_t)v * nrows * 6;
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int b0 = 0; b0 < nrows; b0 += kPoseFinalThreads * kPoseFinalPer) {
        double x[kPoseFinalPer][6];
#pragma unroll
        for (int r = 0; r < kPoseFinalPer; r++) {
            const int b = b0 + r * kPoseFinalThreads + t;
#pragma unroll
            for (int c = 0; c < 6; c++) x[r][c] = b < nrows ? src[(size_t)b * 6 + c] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < kPoseFinalPer; r++)
#pragma unroll
            for (int c = 0; c < 6; c++) s[c] += x[r][c];
    }
    // the 256 x 6 thread sums through LDS in one step: lane 8 c + h of the
    // first wave adds 32 of component c's, then 8-lane shuffles finish
    // (every sum in a fixed order)
#pragma unroll
    for (int c = 0; c < 6; c++) red[c][t] = s[c];
    __syncthreads();
    if (t < 6 * 8) {
        const int c = t >> 3, h = t & 7;
        double x = 0.0;
#pragma unroll 8
        for (int k = 0; k < kPoseFinalThreads / 8; k++) x += red[c][h * (kPoseFinalThreads / 8) + k];
        x += __shfl_xor(x, 1, 8);
        x += __shfl_xor(x, 2, 8);
        x += __shfl_xor(x, 4, 8);
        if (h == 0) {
            const float g = (accumulate ? dpose[6 * v + c] : 0.f) + (float)x;
            dpose[6 * v + c] = g;
            dp6[c] = g;
        }
    }
    if (adam) {
        // the step gsp_pose_adam would take from this gradient (skipped when
        // the render overflowed its instance capacity)
        __syncthreads();
        if (t == 0 && ovf == 0u) {
            double gv[6];
#pragma unroll
            for (int e = 0; e < 6; e++) gv[e] = dp6[e];
            pose_adam_apply(v, k, gv, m0, v0, T0, ad.poses, ad.m, ad.v, ad.steps, ad.p);
        }
    }
}

template <int D>
static void launch_pb(const PbArgs &a, const ViewsK &views, bool want, int nblk, hipStream_t s) {
    if (want)
        hipLaunchKernelGGL((k_preprocess_bwd<D, true>), dim3(nblk), dim3(kPoseReduceBlock), 0, s, a, views);
    else
        hipLaunchKernelGGL((k_preprocess_bwd<D, false>), dim3(nblk), dim3(kPoseReduceBlock), 0, s, a, views);
}

hipError_t launch_preprocess_bwd(const GaussiansK &g, const ViewsK &views, const float *poses,
                                 const Layout &L, char *ws, const gsp_grads &grads,
                                 bool accumulate, hipStream_t s, const PoseAdamK *adam) {
    const bool want = grads.means || grads.scales || grads.quats || grads.opacities || grads.sh;
    PbArgs a;
    a.g = g;
    a.poses = poses;
    a.tiles = region<uint32_t>(ws, L.tiles);
    a.counters = region<uint32_t>(ws, L.counters);
    a.slots = region<float>(ws, L.slots);
    a.grad2d = region<float>(ws, L.grad2d);
    a.posepart = region<double>(ws, L.posepart);
    a.out = grads;
    a.cap = (size_t)L.cap;
    a.vn = (size_t)L.vn;
    a.nblk = L.nblk_pre;
    a.accumulate = accumulate;
    if (L.vn > 0) {
        hipLaunchKernelGGL(k_slot_reduce, dim3(L.nwin_max), dim3(kWindowThreads), 0, s,
                           region<uint32_t>(ws, L.offsets),
                           region<uint2>(ws, L.wstart), a.counters, a.slots,
                           region<uint8_t>(ws, L.slot_flags), a.grad2d,
                           (int)L.vn);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (L.n > 0) {
        switch (g.sh_degree) {
            case 0: launch_pb<0>(a, views, want, L.nblk_pre, s); break;
            case 1: launch_pb<1>(a, views, want, L.nblk_pre, s); break;
            case 2: launch_pb<2>(a, views, want, L.nblk_pre, s); break;
            default: launch_pb<3>(a, views, want, L.nblk_pre, s); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (grads.pose) {
        PoseAdamK ad;
        std::memset(&ad, 0, sizeof ad);
        if (adam) ad = *adam;
        hipLaunchKernelGGL(k_pose_final, dim3(L.V), dim3(kPoseFinalThreads), 0, s, a.posepart,
                           L.nblk_pre * kPoseRowsPerBlock, grads.pose, accumulate, ad,
                           adam != nullptr);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace gsp
