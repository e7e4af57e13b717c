// joint.hip -- the joint reconstruction and pose refinement objective beyond
// the renderer (Sec. III-C): the image loss L_RGB = (1 - beta) L1 +
// beta (1 - SSIM) of Eq. (16) with its gradient, and one Adam step over the
// raw Gaussian parameters with the anisotropy hinge L_An of Eq. (17) folded
// into the scale gradient.
//
// SSIM uses the 11 x 11 Gaussian window (sigma 1.5) of the 3DGS loss the
// paper adopts, C1 = 0.01^2, C2 = 0.03^2 and zero padding outside the image.
// It is computed in two passes over 64 x 16 pixel tiles of one channel: the
// forward filters the five local moments separably (columns first, the
// column sums in LDS) and stores, per pixel, the three partial derivatives
// of SSIM with respect to the filtered quantities (mean, E[x^2], E[xy]); the
// backward filters those three maps with the same (symmetric) window, which
// is the adjoint of the forward filter, and combines them into dL/dpred
// together with the L1 term.  HBM traffic per pixel and channel: x, y in and
// three maps out; three maps, x, y in and the gradient out.
#include "block_ops.h"
#include "gsp_internal.h"

namespace gsp {

constexpr int kSsimR = 5;                        // window radius
constexpr int kSsimTaps = 2 * kSsimR + 1;
constexpr int kSsimTW = 64, kSsimTH = 16;        // output tile
constexpr int kSsimThreads = 256;
constexpr int kSsimLW = kSsimTW + 2 * kSsimR;    // columns with halo
constexpr float kSsimC1 = 0.01f * 0.01f;
constexpr float kSsimC2 = 0.03f * 0.03f;

int ssim_tiles(int w, int h) {
    return ((w + kSsimTW - 1) / kSsimTW) * ((h + kSsimTH - 1) / kSsimTH);
}

__device__ __forceinline__ int rgb_view_of(const RgbViewsK &a, int tile) {
    int v = 0;
    while (v + 1 < a.V && tile >= a.tile_base[v + 1]) v++;
    return v;
}

// Work split of the separable filters, vertical pass first.  A vertical
// work item is one staged column (the 64 output columns plus the 5-column
// halo on each side) and kSsimVR consecutive output rows: it reads its
// kSsimVR + 10 input rows straight from global memory (consecutive threads
// take consecutive columns, so each row is one coalesced segment) and leaves
// the column sums in LDS.  A horizontal item is a run of kSsimHRun outputs
// of one row, read from LDS as aligned vectors.  Each output is still the
// sum over the taps in tap order.  Only the column sums live in LDS (24 KB
// for the forward's five moments), so six blocks fit a CU.
constexpr int kSsimVR = 4;                                   // output rows per vertical item
constexpr int kSsimVIn = kSsimVR + 2 * kSsimR;               // input rows it reads
constexpr int kSsimVItems = kSsimLW * (kSsimTH / kSsimVR);   // 296
constexpr int kSsimHRun = 4;                                 // outputs per horizontal item
constexpr int kSsimHIn = kSsimHRun + 2 * kSsimR;             // column sums it reads
constexpr int kSsimVLD = 76;                                 // row stride of the column sums
static_assert(kSsimTH * (kSsimTW / kSsimHRun) == kSsimThreads, "one horizontal item per thread");
static_assert(kSsimVLD % 4 == 0 && kSsimVLD >= kSsimLW, "16-byte aligned rows");
static_assert(kSsimHIn == 14, "a horizontal item reads three float4 and one float2");

__device__ __forceinline__ void ssim_tile_origin(const RgbViewsK &a, int tile, int &v, int &x0,
                                                 int &y0) {
    v = rgb_view_of(a, tile);
    const int lt = tile - a.tile_base[v];
    x0 = (lt % a.tiles_x[v]) * kSsimTW;
    y0 = (lt / a.tiles_x[v]) * kSsimTH;
}

// The kSsimHIn column sums of a horizontal item, starting at column q0.
__device__ __forceinline__ void ssim_load_run(const float *row, int q0, float (&h)[kSsimHIn]) {
    const float4 a = *reinterpret_cast<const float4 *>(row + q0);
    const float4 b = *reinterpret_cast<const float4 *>(row + q0 + 4);
    const float4 c = *reinterpret_cast<const float4 *>(row + q0 + 8);
    const float2 d = *reinterpret_cast<const float2 *>(row + q0 + 12);
    h[0] = a.x; h[1] = a.y; h[2] = a.z; h[3] = a.w;
    h[4] = b.x; h[5] = b.y; h[6] = b.z; h[7] = b.w;
    h[8] = c.x; h[9] = c.y; h[10] = c.z; h[11] = c.w;
    h[12] = d.x; h[13] = d.y;
}

// partial[c * total_tiles + tile] = (sum of SSIM, sum of |x - y|) of the tile.
__global__ __launch_bounds__(kSsimThreads) void k_ssim_fwd(RgbViewsK a, double2 *partial) {
    __shared__ __align__(16) float vm[5][kSsimTH][kSsimVLD];
    __shared__ double red[kSsimThreads / kWave];
    const int tile = blockIdx.x, c = blockIdx.y;
    int v, x0, y0;
    ssim_tile_origin(a, tile, v, x0, y0);
    const int W = a.w[v], H = a.h[v];
    const size_t plane = (size_t)W * H;
    const float *X = a.pred[v] + c * plane, *Y = a.target[v] + c * plane;
    const int t = threadIdx.x;
    // the L1 sum over the tile's pixels, taken from the vertical items'
    // middle rows (each tile pixel lies in exactly one)
    double l1sum = 0.0;
    for (int item = t; item < kSsimVItems; item += kSsimThreads) {
        const int g = item / kSsimLW, q = item - g * kSsimLW;
        const int gx = x0 + q - kSsimR, gy0 = y0 + kSsimVR * g - kSsimR;
        const bool colin = gx >= 0 && gx < W;
        float xv[kSsimVIn], yv[kSsimVIn];
#pragma unroll
        for (int j = 0; j < kSsimVIn; j++) {
            const int gy = gy0 + j;
            const bool in = colin && gy >= 0 && gy < H;
            xv[j] = in ? X[(size_t)gy * W + gx] : 0.f;
            yv[j] = in ? Y[(size_t)gy * W + gx] : 0.f;
        }
        if (q >= kSsimR && q < kSsimR + kSsimTW && gx < W) {
#pragma unroll
            for (int o = 0; o < kSsimVR; o++)
                if (gy0 + kSsimR + o < H) l1sum += fabs((double)xv[kSsimR + o] - (double)yv[kSsimR + o]);
        }
        // the column's values and their squares and products, once each
        float xx[kSsimVIn], yy[kSsimVIn], xy[kSsimVIn];
#pragma unroll
        for (int j = 0; j < kSsimVIn; j++) {
            xx[j] = xv[j] * xv[j];
            yy[j] = yv[j] * yv[j];
            xy[j] = xv[j] * yv[j];
        }
#pragma unroll
        for (int o = 0; o < kSsimVR; o++) {
            float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
            for (int k = 0; k < kSsimTaps; k++) {
                const float wk = a.win[k];
                s0 = fmaf(wk, xv[o + k], s0);
                s1 = fmaf(wk, yv[o + k], s1);
                s2 = fmaf(wk, xx[o + k], s2);
                s3 = fmaf(wk, yy[o + k], s3);
                s4 = fmaf(wk, xy[o + k], s4);
            }
            const int r = kSsimVR * g + o;
            vm[0][r][q] = s0;
            vm[1][r][q] = s1;
            vm[2][r][q] = s2;
            vm[3][r][q] = s3;
            vm[4][r][q] = s4;
        }
    }
    __syncthreads();
    const int r = t / (kSsimTW / kSsimHRun), q0 = (t % (kSsimTW / kSsimHRun)) * kSsimHRun;
    const int gy = y0 + r;
    float *G = a.gmap[v];
    double ssum = 0.0;
    if (gy < H) {
        float h[5][kSsimHIn];
#pragma unroll
        for (int m = 0; m < 5; m++) ssim_load_run(&vm[m][r][0], q0, h[m]);
        float og[3][kSsimHRun];   // the three maps at the run's pixels
#pragma unroll
        for (int o = 0; o < kSsimHRun; o++) {
            og[0][o] = og[1][o] = og[2][o] = 0.f;
            const int gx = x0 + q0 + o;
            if (gx >= W) continue;
            float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
            for (int k = 0; k < kSsimTaps; k++) {
                const float wk = a.win[k];
                mx = fmaf(wk, h[0][o + k], mx);
                my = fmaf(wk, h[1][o + k], my);
                exx = fmaf(wk, h[2][o + k], exx);
                eyy = fmaf(wk, h[3][o + k], eyy);
                exy = fmaf(wk, h[4][o + k], exy);
            }
            const float sxx = fmaf(-mx, mx, exx), syy = fmaf(-my, my, eyy), sxy = fmaf(-mx, my, exy);
            const float a1 = fmaf(2.f * mx, my, kSsimC1), a2 = fmaf(2.f, sxy, kSsimC2);
            const float b1 = fmaf(mx, mx, fmaf(my, my, kSsimC1)), b2 = sxx + syy + kSsimC2;
            // one division: 1 / b1 = b2 inv and 1 / b2 = b1 inv
            const float inv = __builtin_amdgcn_rcpf(b1 * b2);
            const float S = a1 * a2 * inv;
            // dS/dmu_x, dS/dsigma_x^2, dS/dsigma_xy, then through the raw moments
            const float ds_dmx = 2.f * my * a2 * inv - 2.f * mx * S * (b2 * inv);
            const float ds_dsxx = -S * (b1 * inv);
            const float ds_dsxy = 2.f * a1 * inv;
            og[0][o] = ds_dmx - 2.f * mx * ds_dsxx - my * ds_dsxy;
            og[1][o] = ds_dsxx;
            og[2][o] = ds_dsxy;
            ssum += (double)S;
        }
        const size_t p = (size_t)gy * W + x0 + q0;
        const bool vec = x0 + q0 + kSsimHRun <= W && (p & 3) == 0 && (plane & 3) == 0 &&
                         (reinterpret_cast<uintptr_t>(G) & 15) == 0;
        if (vec) {   // whole 16-byte aligned run: one vector store per map
#pragma unroll
            for (int m = 0; m < 3; m++)
                *reinterpret_cast<float4 *>(G + (size_t)(3 * m + c) * plane + p) =
                    make_float4(og[m][0], og[m][1], og[m][2], og[m][3]);
        } else {
#pragma unroll
            for (int o = 0; o < kSsimHRun; o++)
                if (x0 + q0 + o < W)
#pragma unroll
                    for (int m = 0; m < 3; m++) G[(size_t)(3 * m + c) * plane + p + o] = og[m][o];
        }
    }
    ssum = block_sum<double, kSsimThreads>(ssum, red);
    l1sum = block_sum<double, kSsimThreads>(l1sum, red);
    if (t == 0) partial[(size_t)c * a.total_tiles + tile] = make_double2(ssum, l1sum);
}

// dL/dpred = (1 - beta) sign(x - y) / N - beta / N (F g_mean + 2 x F g_exx +
// y F g_exy), F the window filter (its own adjoint: the window is symmetric
// and the maps are zero outside the image), N = 3 W H.
__global__ __launch_bounds__(kSsimThreads) void k_ssim_bwd(RgbViewsK a) {
    __shared__ __align__(16) float vg[3][kSsimTH][kSsimVLD];
    const int tile = blockIdx.x, c = blockIdx.y;
    int v, x0, y0;
    ssim_tile_origin(a, tile, v, x0, y0);
    const int W = a.w[v], H = a.h[v];
    const size_t plane = (size_t)W * H;
    const float *G = a.gmap[v];
    const int t = threadIdx.x;
    for (int item = t; item < kSsimVItems; item += kSsimThreads) {
        const int g = item / kSsimLW, q = item - g * kSsimLW;
        const int gx = x0 + q - kSsimR, gy0 = y0 + kSsimVR * g - kSsimR;
        const bool colin = gx >= 0 && gx < W;
#pragma unroll
        for (int m = 0; m < 3; m++) {
            const float *Gm = G + (size_t)(3 * m + c) * plane;
            float gv[kSsimVIn];
#pragma unroll
            for (int j = 0; j < kSsimVIn; j++) {
                const int gy = gy0 + j;
                const bool in = colin && gy >= 0 && gy < H;
                gv[j] = in ? Gm[(size_t)gy * W + gx] : 0.f;
            }
#pragma unroll
            for (int o = 0; o < kSsimVR; o++) {
                float s = 0.f;
#pragma unroll
                for (int k = 0; k < kSsimTaps; k++) s = fmaf(a.win[k], gv[o + k], s);
                vg[m][kSsimVR * g + o][q] = s;
            }
        }
    }
    __syncthreads();
    const int r = t / (kSsimTW / kSsimHRun), q0 = (t % (kSsimTW / kSsimHRun)) * kSsimHRun;
    const int gy = y0 + r;
    if (gy >= H) return;
    float h[3][kSsimHIn];
#pragma unroll
    for (int m = 0; m < 3; m++) ssim_load_run(&vg[m][r][0], q0, h[m]);
    const float *X = a.pred[v] + c * plane, *Y = a.target[v] + c * plane;
    float *D = a.grad[v] + c * plane;
    const float invn = 1.f / (3.f * (float)plane);
    const float wl1 = (1.f - a.beta) * invn, wss = -a.beta * invn;
    const size_t p0 = (size_t)gy * W + x0 + q0;
    // whole 16-byte aligned runs move as one vector each
    const bool vec = x0 + q0 + kSsimHRun <= W && (p0 & 3) == 0 && (plane & 3) == 0 &&
                     ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y) |
                       reinterpret_cast<uintptr_t>(D)) & 15) == 0;
    float xs[kSsimHRun], ys[kSsimHRun], ds[kSsimHRun];
    if (vec) {
        const float4 xv = *reinterpret_cast<const float4 *>(X + p0);
        const float4 yv = *reinterpret_cast<const float4 *>(Y + p0);
        xs[0] = xv.x; xs[1] = xv.y; xs[2] = xv.z; xs[3] = xv.w;
        ys[0] = yv.x; ys[1] = yv.y; ys[2] = yv.z; ys[3] = yv.w;
    } else {
#pragma unroll
        for (int o = 0; o < kSsimHRun; o++) {
            const bool in = x0 + q0 + o < W;
            xs[o] = in ? X[p0 + o] : 0.f;
            ys[o] = in ? Y[p0 + o] : 0.f;
        }
    }
#pragma unroll
    for (int o = 0; o < kSsimHRun; o++) {
        float f0 = 0.f, f1 = 0.f, f2 = 0.f;
#pragma unroll
        for (int k = 0; k < kSsimTaps; k++) {
            const float wk = a.win[k];
            f0 = fmaf(wk, h[0][o + k], f0);
            f1 = fmaf(wk, h[1][o + k], f1);
            f2 = fmaf(wk, h[2][o + k], f2);
        }
        const float x = xs[o], y = ys[o];
        const float d = x - y;
        const float sgn = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
        ds[o] = fmaf(wss, fmaf(y, f2, fmaf(2.f * x, f1, f0)), wl1 * sgn);
    }
    if (vec) {
        *reinterpret_cast<float4 *>(D + p0) = make_float4(ds[0], ds[1], ds[2], ds[3]);
    } else {
#pragma unroll
        for (int o = 0; o < kSsimHRun; o++)
            if (x0 + q0 + o < W) D[p0 + o] = ds[o];
    }
}

// One block per view: the view's tile partials in a fixed order.
__global__ __launch_bounds__(256) void k_rgb_final(RgbViewsK a, const double2 *partial,
                                                   float *loss) {
    __shared__ double red[256 / kWave];
    const int v = blockIdx.x;
    const int nt = a.tile_base[v + 1] - a.tile_base[v];
    double s = 0.0, l = 0.0;
    for (int i = threadIdx.x; i < 3 * nt; i += 256) {
        const int c = i / nt, k = i - c * nt;
        const double2 p = partial[(size_t)c * a.total_tiles + a.tile_base[v] + k];
        s += p.x;
        l += p.y;
    }
    s = block_sum<double, 256>(s, red);
    l = block_sum<double, 256>(l, red);
    if (threadIdx.x == 0) {
        const double n = 3.0 * (double)a.w[v] * (double)a.h[v];
        loss[v] = n > 0 ? (float)((1.0 - a.beta) * l / n + a.beta * (1.0 - s / n)) : 0.f;
    }
}

hipError_t launch_loss_rgb(const RgbViewsK &a, float *loss, double2 *partial, hipStream_t s) {
    if (a.total_tiles <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.total_tiles, 3);
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(kSsimThreads), 0, s, a, partial);
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(kSsimThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss) return e;
    hipLaunchKernelGGL(k_rgb_final, dim3(a.V), dim3(256), 0, s, a, partial, loss);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adam over the raw Gaussian parameters.  Work items: one per scalar of the
// means, quaternions, logit opacities and SH coefficients, and one per
// Gaussian for the log scales (all three at once, since the L_An derivative
// of each needs the other two before any is updated).  The update runs in
// FP64 from FP32 storage; the bias corrections and the learning rates come
// from the host.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gauss_adam(GaussAdamK a) {
    __shared__ double red[256 / kWave];
    const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool skip = a.guard && a.guard[kCntOverflow] != 0u;
    double lan = 0.0;
    auto adam = [&](float *p, float *m, float *v, double g, double lr) {
        const double mm = a.b1 * (double)*m + (1.0 - a.b1) * g;
        const double vv = a.b2 * (double)*v + (1.0 - a.b2) * g * g;
        const double np = (double)*p - lr * (mm / a.c1) / (sqrt(vv / a.c2) + a.eps);
        *m = (float)mm;
        *v = (float)vv;
        *p = (float)np;
        return np;
    };
    if (f < a.items[0]) {                       // means: one scalar
        if (!skip) adam(a.means + f, a.m + a.moff[0] + f, a.v + a.moff[0] + f, a.g_means[f], a.lr_means);
    } else if (f < a.items[1]) {                // log scales: one Gaussian
        const int64_t i = f - a.items[0];
        double s[3];
#pragma unroll
        for (int k = 0; k < 3; k++) s[k] = exp((double)a.log_scales[3 * i + k]);
        int imax = 0, imin = 0;
#pragma unroll
        for (int k = 1; k < 3; k++) {
            if (s[k] > s[imax]) imax = k;
            if (s[k] < s[imin]) imin = k;
        }
        const double ratio = s[imax] / s[imin];
        double gan[3] = {0.0, 0.0, 0.0};
        if (ratio > a.aniso_r) {
            lan = ratio - a.aniso_r;
            gan[imax] += 1.0 / (s[imin] * (double)a.n);
            gan[imin] -= s[imax] / (s[imin] * s[imin] * (double)a.n);
        }
        if (!skip) {
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const int64_t e = 3 * i + k;
                const double g = ((double)a.g_scales[e] + a.aniso_w * gan[k]) * s[k];
                const double np = adam(a.log_scales + e, a.m + a.moff[1] + e, a.v + a.moff[1] + e, g,
                                       a.lr_scales);
                a.scales_out[e] = (float)exp(np);
            }
        }
    } else if (f < a.items[2]) {                // quaternions: one scalar
        const int64_t e = f - a.items[1];
        if (!skip) adam(a.quats + e, a.m + a.moff[2] + e, a.v + a.moff[2] + e, a.g_quats[e], a.lr_quats);
    } else if (f < a.items[3]) {                // logit opacities: one scalar
        const int64_t e = f - a.items[2];
        if (!skip) {
            const double o = 1.0 / (1.0 + exp(-(double)a.logits[e]));
            const double g = (double)a.g_opacities[e] * o * (1.0 - o);
            const double np = adam(a.logits + e, a.m + a.moff[3] + e, a.v + a.moff[3] + e, g, a.lr_opacities);
            a.opacities_out[e] = (float)(1.0 / (1.0 + exp(-np)));
        }
    } else if (f < a.items[4]) {                // SH coefficients: one scalar
        const int64_t e = f - a.items[3];
        const int coef = (int)((e / 3) % a.S);
        if (!skip)
            adam(a.sh + e, a.m + a.moff[4] + e, a.v + a.moff[4] + e, a.g_sh[e],
                 coef == 0 ? a.lr_sh_dc : a.lr_sh_rest);
    }
    if (a.partial) {
        // only the blocks that hold log-scale items carry L_An terms
        const int64_t b0 = a.items[0] / 256, b1 = (a.items[1] - 1) / 256;
        if ((int64_t)blockIdx.x >= b0 && (int64_t)blockIdx.x <= b1) {
            lan = block_sum<double, 256>(lan, red);
            if (threadIdx.x == 0) a.partial[blockIdx.x - b0] = lan;
        }
    }
}

__global__ __launch_bounds__(256) void k_aniso_final(const double *partial, int64_t nblk, int64_t n,
                                                     float *loss) {
    __shared__ double red[256 / kWave];
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += 256) s += partial[b];
    s = block_sum<double, 256>(s, red);
    if (threadIdx.x == 0) *loss = n > 0 ? (float)(s / (double)n) : 0.f;
}

int64_t gauss_adam_partials(int64_t n) {
    if (n <= 0) return 0;
    const int64_t items0 = 3 * n, items1 = items0 + n;
    return (items1 - 1) / 256 - items0 / 256 + 1;
}

hipError_t launch_gauss_adam(const GaussAdamK &a, float *aniso_loss, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const int64_t blocks = (a.items[4] + 255) / 256;
    hipLaunchKernelGGL(k_gauss_adam, dim3((unsigned)blocks), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !aniso_loss) return e;
    hipLaunchKernelGGL(k_aniso_final, dim3(1), dim3(256), 0, s, a.partial, gauss_adam_partials(a.n),
                       a.n, aniso_loss);
    return hipGetLastError();
}

}  // namespace gsp
