// misc.hip -- small kernels around the rasterizer: the L1
// photometric loss with its gradient (the L1 part of Eq. (16)), and the
// tangent-space Adam step with left retraction on each pose (Sec. III-B:
// T = Exp(tau), gradients taken on tau).
#include <mutex>

#include "block_ops.h"
#include "gsp_internal.h"
#include "pose_step.h"

namespace gsp {

int64_t loss_blocks(int64_t count) { return (count + kLossItems - 1) / kLossItems; }

// One launch over the views of a call: block b belongs to the view whose block
// range holds it; each view's gradient is normalised by its own value count,
// so a view's loss and gradient do not depend on the other views.
__global__ __launch_bounds__(256) void k_l1(LossViewsK lv, double *partial) {
    __shared__ double red[256 / kWave];
    int v = 0;
    while (v + 1 < lv.V && (int64_t)blockIdx.x >= lv.blk_base[v + 1]) v++;
    const int64_t count = lv.count[v];
    const float *pred = lv.pred[v], *target = lv.target[v];
    float *grad = lv.grad[v];
    const float inv = 1.0f / (float)count;
    const int64_t base = ((int64_t)blockIdx.x - lv.blk_base[v]) * kLossItems;
    double s = 0;
#pragma unroll 4
    for (int r = 0; r < kLossItems / 256; r++) {
        const int64_t k = base + (int64_t)r * 256 + threadIdx.x;
        if (k < count) {
            const float d = pred[k] - target[k];
            grad[k] = d > 0.f ? inv : (d < 0.f ? -inv : 0.f);
            s += fabs((double)d);
        }
    }
    if (partial) {
        s = block_sum<double, 256>(s, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// One block per view: the view's partial sums in block order.
__global__ __launch_bounds__(256) void k_l1_final(LossViewsK lv, const double *partial,
                                                  float *loss) {
    __shared__ double red[256 / kWave];
    const int v = blockIdx.x;
    double s = 0;
    for (int64_t b = lv.blk_base[v] + threadIdx.x; b < lv.blk_base[v + 1]; b += 256) s += partial[b];
    s = block_sum<double, 256>(s, red);
    if (threadIdx.x == 0) loss[v] = (float)(s / (double)lv.count[v]);
}

// Scratch of gsp_loss_l1_noalloc: the per-block partial sums of the loss,
// in a fixed array of the library instead of caller memory.  Each device
// that loads the library holds its own copy until the process ends.  Host
// code must not pass the array's name to a kernel (on the host it is only a
// stand-in for the device symbol): its device address comes from
// hipGetSymbolAddress, taken once per device by noalloc_scratch_init.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
void *g_noalloc_ptr[kMaxDevices];
bool g_noalloc_done[kMaxDevices];
std::mutex g_noalloc_mutex;
}  // namespace

hipError_t noalloc_scratch_init(int device, void **ptr) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    if (!g_noalloc_done[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if ((e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t e2 = hipSetDevice(prev);
        if (e != hipSuccess) return e;
        if (e2 != hipSuccess) return e2;
        g_noalloc_ptr[device] = p;
        g_noalloc_done[device] = true;
    }
    *ptr = g_noalloc_ptr[device];
    return hipSuccess;
}

hipError_t launch_loss_l1(const LossViewsK &lv, float *loss, void *partial_buf, hipStream_t s) {
    const int64_t nblk = lv.blk_base[lv.V];
    if (nblk <= 0) return hipSuccess;
    double *partial = loss ? static_cast<double *>(partial_buf) : nullptr;
    hipLaunchKernelGGL(k_l1, dim3((unsigned)nblk), dim3(256), 0, s, lv, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss) return e;
    hipLaunchKernelGGL(k_l1_final, dim3(lv.V), dim3(256), 0, s, lv, partial, loss);
    return hipGetLastError();
}

// guard: the counters of the workspace whose render produced dpose, or null;
// when that render overflowed its instance capacity the step is skipped
// (poses, moments and step counts unchanged).
__global__ __launch_bounds__(64) void k_pose_adam(int V, float *poses, const float *dpose, float *m,
                                                  float *v, int32_t *steps, gsp_adam_params p,
                                                  const uint32_t *guard) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= V) return;
    // every load first (one round of memory latency), then the guard test
    const uint32_t ovf = guard ? guard[kCntOverflow] : 0u;
    const int k = steps[i] + 1;
    double gv[6], m0[6], v0[6];
    float T0[12];
#pragma unroll
    for (int e = 0; e < 6; e++) {
        gv[e] = dpose[6 * i + e];
        m0[e] = m[6 * i + e];
        v0[e] = v[6 * i + e];
    }
#pragma unroll
    for (int e = 0; e < 12; e++) T0[e] = poses[12 * i + e];
    if (ovf != 0u) return;
    pose_adam_apply(i, k, gv, m0, v0, T0, poses, m, v, steps, p);
}

hipError_t launch_pose_adam(int V, float *poses, const float *dpose, float *m, float *v,
                            int32_t *steps, const gsp_adam_params &p, const uint32_t *guard,
                            hipStream_t s) {
    if (V <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pose_adam, dim3((V + 63) / 64), dim3(64), 0, s, V, poses, dpose, m, v, steps, p,
                       guard);
    return hipGetLastError();
}

// T' = Exp(tau) T per view: the pose a twist tau moves the world->camera
// pose T to under the left perturbation of Sec. III-B (FP64, stored FP32).
__global__ __launch_bounds__(64) void k_twist_apply(int V, const float *tau, const float *poses,
                                                    float *out) {
    const int v = blockIdx.x * 64 + threadIdx.x;
    if (v >= V) return;
    double d[6];
    for (int k = 0; k < 6; k++) d[k] = tau[6 * v + k];
    float T[12];
    for (int k = 0; k < 12; k++) T[k] = poses[12 * v + k];
    se3_retract_left(d, T);
    for (int k = 0; k < 12; k++) out[12 * v + k] = T[k];
}

// dL/dtau at tau from the twist gradient g at T' = Exp(tau) T: since
// Exp(tau + delta) = Exp(J(tau) delta) Exp(tau) to first order, with J the
// left Jacobian of SE(3) for tau = (rho, phi),
//   J = [[Jr, Q], [0, Jr]],  Jr = I + b [phi]x + c [phi]x^2,
//   Q = 1/2 [rho]x + c (P R + R P + P R P) + e (P P R + R P P - 3 P R P)
//       + f (P R P P + P P R P),   P = [phi]x, R = [rho]x,
// b = (1 - cos t) / t^2, c = (t - sin t) / t^3, e = (t^2/2 + cos t - 1) / t^4,
// f = (e + 3 (t - sin t - t^3/6) / t^5) / 2, t = |phi| (series below 1e-2),
// the gradient is J^T g: (Jr^T g_rho, Q^T g_rho + Jr^T g_phi).
__device__ void mat3_mul_d(const double *A, const double *B, double *C) {
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++)
            C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

__global__ __launch_bounds__(64) void k_twist_chain(int V, const float *tau, const float *g,
                                                    float *out) {
    const int v = blockIdx.x * 64 + threadIdx.x;
    if (v >= V) return;
    const double r0 = tau[6 * v], r1 = tau[6 * v + 1], r2 = tau[6 * v + 2];
    const double p0 = tau[6 * v + 3], p1 = tau[6 * v + 4], p2 = tau[6 * v + 5];
    const double t2 = p0 * p0 + p1 * p1 + p2 * p2, t = sqrt(t2);
    double b, c, e, f;
    if (t < 1e-2) {
        b = 0.5 - t2 / 24 + t2 * t2 / 720;
        c = 1.0 / 6 - t2 / 120 + t2 * t2 / 5040;
        e = 1.0 / 24 - t2 / 720 + t2 * t2 / 40320;
        const double h = -1.0 / 120 + t2 / 5040 - t2 * t2 / 362880;   // (t - sin t - t^3/6) / t^5
        f = 0.5 * (e + 3.0 * h);
    } else {
        const double st = sin(t), ct = cos(t);
        b = (1 - ct) / t2;
        c = (t - st) / (t2 * t);
        e = (0.5 * t2 + ct - 1) / (t2 * t2);
        f = 0.5 * (e + 3.0 * (t - st - t2 * t / 6) / (t2 * t2 * t));
    }
    const double P[9] = {0, -p2, p1, p2, 0, -p0, -p1, p0, 0};
    const double R[9] = {0, -r2, r1, r2, 0, -r0, -r1, r0, 0};
    double PP[9], PR[9], RP[9], PRP[9], PPR[9], RPP[9], PRPP[9], PPRP[9];
    mat3_mul_d(P, P, PP);
    mat3_mul_d(P, R, PR);
    mat3_mul_d(R, P, RP);
    mat3_mul_d(PR, P, PRP);
    mat3_mul_d(PP, R, PPR);
    mat3_mul_d(RP, P, RPP);
    mat3_mul_d(PRP, P, PRPP);
    mat3_mul_d(PP, RP, PPRP);
    double Jr[9], Q[9];
    for (int k = 0; k < 9; k++) {
        Jr[k] = (k % 4 == 0 ? 1.0 : 0.0) + b * P[k] + c * PP[k];
        Q[k] = 0.5 * R[k] + c * (PR[k] + RP[k] + PRP[k]) + e * (PPR[k] + RPP[k] - 3.0 * PRP[k]) +
               f * (PRPP[k] + PPRP[k]);
    }
    double gr[3], gp[3];
    for (int k = 0; k < 3; k++) {
        gr[k] = g[6 * v + k];
        gp[k] = g[6 * v + 3 + k];
    }
    for (int k = 0; k < 3; k++) {
        double a = 0, q = 0;
        for (int i = 0; i < 3; i++) {
            a += Jr[3 * i + k] * gr[i];
            q += Q[3 * i + k] * gr[i] + Jr[3 * i + k] * gp[i];
        }
        out[6 * v + k] = (float)a;
        out[6 * v + 3 + k] = (float)q;
    }
}

hipError_t launch_twist_apply(int V, const float *tau, const float *poses, float *out,
                              hipStream_t s) {
    if (V <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_twist_apply, dim3((V + 63) / 64), dim3(64), 0, s, V, tau, poses, out);
    return hipGetLastError();
}

hipError_t launch_twist_chain(int V, const float *tau, const float *g, float *out, hipStream_t s) {
    if (V <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_twist_chain, dim3((V + 63) / 64), dim3(64), 0, s, V, tau, g, out);
    return hipGetLastError();
}

}  // namespace gsp
