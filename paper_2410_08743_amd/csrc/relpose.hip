// relpose.hip -- relative pose estimation between two frames (Sec. III-D):
// the scene of frame t from its depth map (pixels on a stride grid
// unprojected through the intrinsics into isotropic Gaussians with the
// pixel's colour and, as scale, the mean distance to their three nearest
// neighbours), and the confidence-masked L1 of Eq. (20)-(21) that the pose
// of frame t+1 is solved against.
//
// The nearest neighbours are found by brute force: every query thread walks
// all points in LDS tiles of 256 (broadcast reads) and keeps its three
// smallest squared distances with a branch-free min/max insertion.  At the
// sizes the method uses (tens of thousands of points) this is a few
// milliseconds of FP32 ALU work and needs no spatial structure.
#include "block_ops.h"
#include "gsp_internal.h"

namespace gsp {

constexpr float kY0 = 0.28209479177387814f;   // degree-0 SH basis value
constexpr float kInvalidLogit = -30.f;        // opacity of a pixel without depth
constexpr float kInvalidScale = 0.01f;        // scale of a point without neighbours
constexpr int kKnnThreads = 256;

__global__ __launch_bounds__(256) void k_unproject(UnprojK a) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    const int n = a.nx * a.ny;
    if (k >= n) return;
    const int x = (k % a.nx) * a.stride, y = (k / a.nx) * a.stride;
    const size_t pix = (size_t)y * a.w + x;
    const float d = a.depth[pix];
    const bool ok = isfinite(d) && d > 0.f;
    const float z = ok ? d : 1.f;
    const float X = ((float)(x + a.roi_x) + 0.5f - a.cx) / a.fx * z;
    const float Y = ((float)(y + a.roi_y) + 0.5f - a.cy) / a.fy * z;
    a.means[3 * (size_t)k] = X;
    a.means[3 * (size_t)k + 1] = Y;
    a.means[3 * (size_t)k + 2] = z;
    a.quats[4 * (size_t)k] = 1.f;
    a.quats[4 * (size_t)k + 1] = 0.f;
    a.quats[4 * (size_t)k + 2] = 0.f;
    a.quats[4 * (size_t)k + 3] = 0.f;
    a.logits[k] = ok ? a.logit : kInvalidLogit;
    const size_t plane = (size_t)a.w * a.h;
    float *sh = a.sh + (size_t)k * 3 * a.S;
#pragma unroll
    for (int c = 0; c < 3; c++) sh[c] = (a.image[c * plane + pix] - 0.5f) / kY0;
    for (int e = 3; e < 3 * a.S; e++) sh[e] = 0.f;
    a.pts[k] = make_float4(X, Y, z, ok ? 1.f : 0.f);
}

// log of the mean distance of each point to its three nearest valid
// neighbours (itself excluded), written to all three log scales.
__global__ __launch_bounds__(kKnnThreads) void k_knn3(const float4 *pts, int n, float *log_scales) {
    __shared__ float4 tile[kKnnThreads];
    const int k = blockIdx.x * kKnnThreads + threadIdx.x;
    const float4 q = k < n ? pts[k] : make_float4(0.f, 0.f, 0.f, 0.f);
    float b0 = INFINITY, b1 = INFINITY, b2 = INFINITY;
    for (int base = 0; base < n; base += kKnnThreads) {
        const int c = base + (int)threadIdx.x;
        tile[threadIdx.x] = c < n ? pts[c] : make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        const int cnt = min(kKnnThreads, n - base);
        for (int j = 0; j < cnt; j++) {
            const float4 p = tile[j];
            const float dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
            float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            d2 = (p.w != 0.f && base + j != k) ? d2 : INFINITY;
            // insert into the sorted triple b0 <= b1 <= b2
            const float n0 = fminf(b0, d2);
            const float n1 = fminf(b1, fmaxf(b0, d2));
            const float n2 = fminf(b2, fmaxf(b1, d2));
            b0 = n0;
            b1 = n1;
            b2 = n2;
        }
        __syncthreads();
    }
    if (k >= n) return;
    float sum = 0.f;
    int cnt = 0;
    if (b0 < INFINITY) { sum += sqrtf(b0); cnt++; }
    if (b1 < INFINITY) { sum += sqrtf(b1); cnt++; }
    if (b2 < INFINITY) { sum += sqrtf(b2); cnt++; }
    const float ls = logf(cnt > 0 ? sum / (float)cnt : kInvalidScale);
    log_scales[3 * (size_t)k] = ls;
    log_scales[3 * (size_t)k + 1] = ls;
    log_scales[3 * (size_t)k + 2] = ls;
}

hipError_t launch_unproject(const UnprojK &a, hipStream_t s) {
    const int n = a.nx * a.ny;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unproject, dim3((n + 255) / 256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_knn3, dim3((n + kKnnThreads - 1) / kKnnThreads), dim3(kKnnThreads), 0, s,
                       a.pts, n, a.log_scales);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Masked L1 (Eq. (21)): loss[v] = sum over pixels and channels of
// M |pred - target|, grad = M sign(pred - target), M = [alpha > 0.99] with
// alpha = 1 - T_final the render's accumulated opacity (Eq. (20)); the mask
// is decided in FP64 on the FP32 alpha.
// ---------------------------------------------------------------------------
constexpr int kMaskItems = 4096;

int64_t masked_blocks(int64_t count) { return (count + kMaskItems - 1) / kMaskItems; }

__global__ __launch_bounds__(256) void k_masked_l1(MaskViewsK a, double *partial) {
    __shared__ double red[256 / kWave];
    int v = 0;
    while (v + 1 < a.V && (int64_t)blockIdx.x >= a.blk_base[v + 1]) v++;
    const int64_t P = a.pix[v], count = 3 * P;
    const float *pred = a.pred[v], *target = a.target[v], *alpha = a.alpha[v];
    float *grad = a.grad[v];
    const int64_t base = ((int64_t)blockIdx.x - a.blk_base[v]) * kMaskItems;
    double s = 0.0;
#pragma unroll 4
    for (int r = 0; r < kMaskItems / 256; r++) {
        const int64_t e = base + (int64_t)r * 256 + threadIdx.x;
        if (e < count) {
            const bool m = (double)alpha[e % P] > 0.99;
            const float d = pred[e] - target[e];
            grad[e] = m ? (d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f)) : 0.f;
            s += m ? fabs((double)d) : 0.0;
        }
    }
    if (partial) {
        s = block_sum<double, 256>(s, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void k_masked_l1_final(MaskViewsK a, const double *partial,
                                                         float *loss) {
    __shared__ double red[256 / kWave];
    const int v = blockIdx.x;
    double s = 0.0;
    for (int64_t b = a.blk_base[v] + threadIdx.x; b < a.blk_base[v + 1]; b += 256) s += partial[b];
    s = block_sum<double, 256>(s, red);
    if (threadIdx.x == 0) loss[v] = (float)s;
}

hipError_t launch_masked_l1(const MaskViewsK &a, float *loss, void *scratch, hipStream_t s) {
    const int64_t nblk = a.blk_base[a.V];
    if (nblk <= 0) return hipSuccess;
    double *partial = loss ? static_cast<double *>(scratch) : nullptr;
    hipLaunchKernelGGL(k_masked_l1, dim3((unsigned)nblk), dim3(256), 0, s, a, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss) return e;
    hipLaunchKernelGGL(k_masked_l1_final, dim3(a.V), dim3(256), 0, s, a, partial, loss);
    return hipGetLastError();
}

}  // namespace gsp
