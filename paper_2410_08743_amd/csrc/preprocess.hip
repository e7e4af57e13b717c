// preprocess.hip -- projection of every Gaussian into every view of a call,
// and duplication of each projected splat into (tile | depth) sort keys.
//
// Sec. III-A: Sigma = R(q) diag(s)^2 R(q)^T (Eq. (1)); mu_hat = pi(K T mu);
// Sigma_hat = [J R_c Sigma R_c^T J^T]_2x2 (Eq. (2)) plus a 0.3 px^2
// dilation; colour = SH(f, d) with d = (mu - o_c) / |mu - o_c|,
// o_c = -R_c^T t_c.
//
// MI355X design: one thread per Gaussian reads the parameters once and loops
// over the call's views (one HBM read of the 236 B/Gaussian SH-3 record per
// call, however many views).  Geometry is computed in FP64 -- the vector
// FP64 rate of gfx950 is that of unpacked FP32 and this kernel is bound by
// HBM, so the extra precision is free -- and the projected centre is stored
// as an FP32 (hi, lo) pair so that the rasterizer can form pixel offsets to
// ~1e-6 px.  The sort key's depth is float32 of the camera-frame z computed
// by a fixed FMA chain, which makes keys reproducible bit for bit.
#include "block_ops.h"
#include "gsp_internal.h"
#include "sh_basis.h"

namespace gsp {

struct PreArgs {
    GaussiansK g;
    const float *poses;
    float4 *geom;                  // [vn][2]: (u_hi, v_hi, u_lo, v_lo), (A2, B2, C2, log2 o)
    float4 *color;                 // [vn]: (r, g, b, 0)
    uint2 *rect;                   // [vn]: x0 | y0 << 16, x1 | y1 << 16
    uint32_t *depth;               // [vn]: float bits of the key depth
    uint32_t *tiles;               // [vn]: tiles touched
    uint32_t *dkeys;               // [vn]: depth-sort key (depth bits; ~0 when not drawn)
    uint32_t *dvals;               // [vn]: view * n + i
};

template <int D>
__global__ __launch_bounds__(kPreprocessBlock) void k_preprocess(PreArgs a, ViewsK views) {
    constexpr int S = (D + 1) * (D + 1);
    const int n = a.g.n;
    const int i = blockIdx.x * kPreprocessBlock + threadIdx.x;
    const bool valid = i < n;

    double mu[3] = {0, 0, 0};
    double Sig[6] = {0, 0, 0, 0, 0, 0};  // xx xy xz yy yz zz
    float opac = 0.f;
    float sh[S * 3];
#pragma unroll
    for (int k = 0; k < S * 3; k++) sh[k] = 0.f;
    if (valid) {
        mu[0] = a.g.means[3 * i];
        mu[1] = a.g.means[3 * i + 1];
        mu[2] = a.g.means[3 * i + 2];
        const double s0 = a.g.scales[3 * i], s1 = a.g.scales[3 * i + 1],
                     s2 = a.g.scales[3 * i + 2];
        double qw = a.g.quats[4 * i], qx = a.g.quats[4 * i + 1], qy = a.g.quats[4 * i + 2],
               qz = a.g.quats[4 * i + 3];
        const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        qw /= qn; qx /= qn; qy /= qn; qz /= qn;
        // rotation of the unit quaternion (w, x, y, z)
        const double r00 = 1 - 2 * (qy * qy + qz * qz), r01 = 2 * (qx * qy - qw * qz),
                     r02 = 2 * (qx * qz + qw * qy);
        const double r10 = 2 * (qx * qy + qw * qz), r11 = 1 - 2 * (qx * qx + qz * qz),
                     r12 = 2 * (qy * qz - qw * qx);
        const double r20 = 2 * (qx * qz - qw * qy), r21 = 2 * (qy * qz + qw * qx),
                     r22 = 1 - 2 * (qx * qx + qy * qy);
        const double e0 = s0 * s0, e1 = s1 * s1, e2 = s2 * s2;
        Sig[0] = r00 * r00 * e0 + r01 * r01 * e1 + r02 * r02 * e2;
        Sig[1] = r00 * r10 * e0 + r01 * r11 * e1 + r02 * r12 * e2;
        Sig[2] = r00 * r20 * e0 + r01 * r21 * e1 + r02 * r22 * e2;
        Sig[3] = r10 * r10 * e0 + r11 * r11 * e1 + r12 * r12 * e2;
        Sig[4] = r10 * r20 * e0 + r11 * r21 * e1 + r12 * r22 * e2;
        Sig[5] = r20 * r20 * e0 + r21 * r21 * e1 + r22 * r22 * e2;
        opac = a.g.opacities[i];
        const float *f = a.g.sh + (size_t)i * (S * 3);
#pragma unroll
        for (int k = 0; k < S * 3; k++) sh[k] = f[k];
    }

    for (int v = 0; v < views.count; v++) {
        const ViewK &vw = views.v[v];
        const float *P = a.poses + 12 * v;
        const size_t idx = (size_t)v * n + i;
        uint32_t cnt = 0;
        if (valid) {
            double R[9], t[3];
#pragma unroll
            for (int r = 0; r < 3; r++) {
                R[3 * r] = P[4 * r];
                R[3 * r + 1] = P[4 * r + 1];
                R[3 * r + 2] = P[4 * r + 2];
                t[r] = P[4 * r + 3];
            }
            double p[3];
#pragma unroll
            for (int r = 0; r < 3; r++)
                p[r] = fma(R[3 * r + 2], mu[2], fma(R[3 * r + 1], mu[1], fma(R[3 * r], mu[0], t[r])));
            const float zkey = (float)p[2];
            uint2 rect = make_uint2(0, 0);
            float4 g0 = make_float4(0, 0, 0, 0), g1 = make_float4(0, 0, 0, 0);
            float4 col = make_float4(0, 0, 0, 0);
            const double z = p[2];
            bool keep = z > kNear;
            double u = 0, vv = 0, A = 0, B = 0, C = 0;
            if (keep) {
                u = vw.fx * p[0] / z + vw.cx - 0.5;
                vv = vw.fy * p[1] / z + vw.cy - 0.5;
                const double limx = kJClamp * 0.5 * vw.W / (double)vw.fx;
                const double limy = kJClamp * 0.5 * vw.H / (double)vw.fy;
                const double xz = fmin(fmax(p[0] / z, -limx), limx);
                const double yz = fmin(fmax(p[1] / z, -limy), limy);
                const double j00 = vw.fx / z, j02 = -vw.fx * xz / z;
                const double j11 = vw.fy / z, j12 = -vw.fy * yz / z;
                // T2 = J R_c (2 x 3)
                const double a0 = j00 * R[0] + j02 * R[6], a1 = j00 * R[1] + j02 * R[7],
                             a2 = j00 * R[2] + j02 * R[8];
                const double b0 = j11 * R[3] + j12 * R[6], b1 = j11 * R[4] + j12 * R[7],
                             b2 = j11 * R[5] + j12 * R[8];
                // Sigma * t for both rows
                const double sa0 = Sig[0] * a0 + Sig[1] * a1 + Sig[2] * a2;
                const double sa1 = Sig[1] * a0 + Sig[3] * a1 + Sig[4] * a2;
                const double sa2 = Sig[2] * a0 + Sig[4] * a1 + Sig[5] * a2;
                const double sb0 = Sig[0] * b0 + Sig[1] * b1 + Sig[2] * b2;
                const double sb1 = Sig[1] * b0 + Sig[3] * b1 + Sig[4] * b2;
                const double sb2 = Sig[2] * b0 + Sig[4] * b1 + Sig[5] * b2;
                const double ca = a0 * sa0 + a1 * sa1 + a2 * sa2 + kDilation;
                const double cb = a0 * sb0 + a1 * sb1 + a2 * sb2;
                const double cc = b0 * sb0 + b1 * sb1 + b2 * sb2 + kDilation;
                const double det = ca * cc - cb * cb;
                keep = det > 0;
                if (keep) {
                    A = cc / det;
                    B = -cb / det;
                    C = ca / det;
                    const double mid = 0.5 * (ca + cc);
                    const double lam = mid + sqrt(fmax(mid * mid - det, kLambdaFloor));
                    const double r = ceil(3.0 * sqrt(lam));
                    const int ox = vw.roi_x / kTile, oy = vw.roi_y / kTile;
                    const double x0 = fmin(fmax(floor((u - r) / kTile) - ox, 0.0), (double)vw.gw);
                    const double x1 = fmin(fmax(floor((u + r + kTile - 1) / kTile) - ox, 0.0), (double)vw.gw);
                    const double y0 = fmin(fmax(floor((vv - r) / kTile) - oy, 0.0), (double)vw.gh);
                    const double y1 = fmin(fmax(floor((vv + r + kTile - 1) / kTile) - oy, 0.0), (double)vw.gh);
                    const uint32_t ix0 = (uint32_t)x0, ix1 = (uint32_t)x1, iy0 = (uint32_t)y0,
                                   iy1 = (uint32_t)y1;
                    cnt = (ix1 - ix0) * (iy1 - iy0);
                    rect = make_uint2(ix0 | (iy0 << 16), ix1 | (iy1 << 16));
                }
            }
            if (cnt > 0) {
                const float uh = (float)u, vh = (float)vv;
                g0 = make_float4(uh, vh, (float)(u - (double)uh), (float)(vv - (double)vh));
                // conic in base 2 with the -1/2 folded in, and log2 of the opacity
                g1 = make_float4((float)(-0.5 * kLog2e * A), (float)(-kLog2e * B),
                                 (float)(-0.5 * kLog2e * C), (float)log2((double)opac));
                // camera centre o_c = -R^T t and the viewing direction
                const double ocx = -(R[0] * t[0] + R[3] * t[1] + R[6] * t[2]);
                const double ocy = -(R[1] * t[0] + R[4] * t[1] + R[7] * t[2]);
                const double ocz = -(R[2] * t[0] + R[5] * t[1] + R[8] * t[2]);
                double dx = mu[0] - ocx, dy = mu[1] - ocy, dz = mu[2] - ocz;
                const double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
                float Y[S];
                sh_eval<D, float>((float)(dx * inv), (float)(dy * inv), (float)(dz * inv), Y);
                float c3[3];
#pragma unroll
                for (int ch = 0; ch < 3; ch++) {
                    float acc = 0.f;
#pragma unroll
                    for (int k = 0; k < S; k++) acc = fmaf(sh[3 * k + ch], Y[k], acc);
                    c3[ch] = fmaxf(acc + 0.5f, 0.f);
                }
                col = make_float4(c3[0], c3[1], c3[2], 0.f);
            }
            a.geom[2 * idx] = g0;
            a.geom[2 * idx + 1] = g1;
            a.color[idx] = col;
            a.rect[idx] = rect;
            a.depth[idx] = __float_as_uint(zkey);
            a.tiles[idx] = cnt;
            a.dkeys[idx] = cnt > 0 ? __float_as_uint(zkey) : 0xffffffffu;
            a.dvals[idx] = (uint32_t)idx;
        }
    }
}

// Per-block sums of the tile counts, taken in depth order.
__global__ __launch_bounds__(kPreprocessBlock) void k_sorted_blocksums(const uint32_t *order,
                                                                       const uint32_t *tiles,
                                                                       unsigned long long *bs,
                                                                       int vn) {
    __shared__ unsigned long long red[kPreprocessBlock / kWave];
    const int k = blockIdx.x * kPreprocessBlock + threadIdx.x;
    const uint32_t cnt = k < vn ? tiles[order[k]] : 0u;
    const unsigned long long s = block_sum<unsigned long long, kPreprocessBlock>(cnt, red);
    if (threadIdx.x == 0) bs[blockIdx.x] = s;
}

// Exclusive scan of the per-(view, block) instance counts in one block; the
// grand total is M.  Writes M, the overflow flag and the effective M (0 on
// overflow, so that every later stage does no work).
__global__ __launch_bounds__(1024) void k_scan_blocksums(unsigned long long *bs, int count,
                                                         uint32_t *counters,
                                                         unsigned long long cap) {
    __shared__ unsigned long long scratch[1024 / kWave];
    const int t = threadIdx.x;
    const int per = (count + 1023) / 1024;
    const int begin = min(t * per, count), end = min(begin + per, count);
    unsigned long long local = 0;
    for (int k = begin; k < end; k++) local += bs[k];
    unsigned long long total;
    unsigned long long off = block_exclusive_scan<unsigned long long, 1024>(local, scratch, &total);
    for (int k = begin; k < end; k++) {
        const unsigned long long x = bs[k];
        bs[k] = off;
        off += x;
    }
    if (t == 0) {
        const bool ovf = total > cap;
        counters[kCntMLo] = (uint32_t)(total & 0xffffffffull);
        counters[kCntMHi] = (uint32_t)(total >> 32);
        counters[kCntOverflow] = ovf ? 1u : 0u;
        counters[kCntMEff] = ovf ? 0u : (uint32_t)total;
        if (ovf) counters[kCntSticky] = 1u;
    }
}

struct DupArgs {
    const uint32_t *order;         // [vn] view * n + i in (depth, index) order
    const uint2 *rect;
    const uint32_t *tiles;
    uint32_t *offsets;             // [vn] by splat: first emission position
    uint32_t *offk;                // [vn + 1] by depth rank: first emission position, then M
    uint32_t *wstart;              // [windows + 1] first depth rank of each work window
    const unsigned long long *blockoff;
    uint32_t *counters;
    uint32_t *keys;
    uint32_t *vals;
    int vn;
};

// Exclusive offsets of the splats' instance runs in depth order, and the
// work windows.  Splat k's entry sits at position h = k + offk[k] of the
// sequence (splat, its instances, next splat, ...), the next at h + 1 + cnt;
// window b starts at the first splat whose entry is at or after b * kWindow.
__global__ __launch_bounds__(kPreprocessBlock) void k_offsets(DupArgs a) {
    __shared__ unsigned long long scratch[kPreprocessBlock / kWave];
    const int k = blockIdx.x * kPreprocessBlock + threadIdx.x;
    const uint32_t idx = k < a.vn ? a.order[k] : 0u;
    const uint32_t cnt = k < a.vn ? a.tiles[idx] : 0u;
    unsigned long long total;
    const unsigned long long excl =
        block_exclusive_scan<unsigned long long, kPreprocessBlock>(cnt, scratch, &total) +
        a.blockoff[blockIdx.x];
    if (a.counters[kCntOverflow] != 0u || k >= a.vn) return;
    a.offsets[idx] = (uint32_t)excl;
    a.offk[k] = (uint32_t)excl;
    const unsigned long long h = (unsigned long long)k + excl, h1 = h + 1 + cnt;
    if (k == 0) a.wstart[0] = 0u;
    for (unsigned long long b = h / kWindow + 1; b * kWindow <= h1; b++) a.wstart[b] = (uint32_t)k + 1;
    if (k == a.vn - 1) {
        const unsigned long long nwin = (h1 + kWindow - 1) / kWindow;
        if (nwin * kWindow > h1) a.wstart[nwin] = (uint32_t)a.vn;
        a.offk[a.vn] = (uint32_t)(excl + cnt);
        a.counters[kCntWin] = (uint32_t)nwin;
    }
}

// Emits one (tile, view * n + i) pair per tile of each splat's rect, rows
// outer and columns inner, at the splat's offset; a stable sort of these
// pairs by tile then yields every tile's list in (depth, index) order.  One
// block per work window; each thread writes consecutive positions and finds
// the splat owning a position by binary search over the window's offsets.
__global__ __launch_bounds__(kWindowThreads) void k_emit(DupArgs a, ViewsK views, int n) {
    __shared__ uint32_t s_off[kWindow + 1];
    __shared__ uint32_t s_idx[kWindow];
    __shared__ uint2 s_rect[kWindow];
    const int b = blockIdx.x;
    if (a.counters[kCntOverflow] != 0u || (uint32_t)b >= a.counters[kCntWin]) return;
    const uint32_t kb = a.wstart[b], ke = a.wstart[b + 1];
    const int nk = (int)(ke - kb);   // at most kWindow
    for (int j = threadIdx.x; j < nk; j += kWindowThreads) {
        const uint32_t idx = a.order[kb + j];
        s_off[j] = a.offk[kb + j];
        s_idx[j] = idx;
        s_rect[j] = a.rect[idx];
    }
    const uint32_t e0 = a.offk[kb], e1 = a.offk[ke];
    if (threadIdx.x == 0) s_off[nk] = e1;
    __syncthreads();
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += kWindowThreads) {
        // largest j with s_off[j] <= e; s_off[0] <= e < s_off[nk]
        int lo = 0, hi = nk;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_off[mid] <= e) lo = mid; else hi = mid;
        }
        const uint2 r = s_rect[lo];
        const int x0 = r.x & 0xffff, y0 = r.x >> 16, x1 = r.y & 0xffff;
        const uint32_t w = (uint32_t)(x1 - x0), local = e - s_off[lo];
        const uint32_t idx = s_idx[lo];
        const ViewK &vw = views.v[idx / (uint32_t)n];
        const uint32_t ty = (uint32_t)y0 + local / w, tx = (uint32_t)x0 + local % w;
        a.keys[e] = (uint32_t)vw.tile_base + ty * (uint32_t)vw.gw + tx;
        a.vals[e] = idx;
    }
}

hipError_t launch_preprocess(const GaussiansK &g, const ViewsK &views, const float *poses,
                             const Layout &L, char *ws, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    PreArgs a;
    a.g = g;
    a.poses = poses;
    a.geom = region<float4>(ws, L.geom);
    a.color = region<float4>(ws, L.color);
    a.rect = region<uint2>(ws, L.rect);
    a.depth = region<uint32_t>(ws, L.depth);
    a.tiles = region<uint32_t>(ws, L.tiles);
    a.dkeys = region<uint32_t>(ws, L.dkeys0);
    a.dvals = region<uint32_t>(ws, L.dvals0);
    dim3 grid(L.nblk_pre), block(kPreprocessBlock);
    switch (g.sh_degree) {
        case 0: hipLaunchKernelGGL(k_preprocess<0>, grid, block, 0, s, a, views); break;
        case 1: hipLaunchKernelGGL(k_preprocess<1>, grid, block, 0, s, a, views); break;
        case 2: hipLaunchKernelGGL(k_preprocess<2>, grid, block, 0, s, a, views); break;
        default: hipLaunchKernelGGL(k_preprocess<3>, grid, block, 0, s, a, views); break;
    }
    return hipGetLastError();
}

hipError_t launch_offsets_and_duplicate(const ViewsK &views, const Layout &L, char *ws,
                                        hipStream_t s) {
    unsigned long long *bs = region<unsigned long long>(ws, L.blocksum);
    uint32_t *counters = region<uint32_t>(ws, L.counters);
    const uint32_t *order = region<uint32_t>(ws, L.dvals0);   // depth sort: 4 passes, even
    const int vn = (int)L.vn;
    if (vn > 0) {
        hipLaunchKernelGGL(k_sorted_blocksums, dim3(L.nblk_vn), dim3(kPreprocessBlock), 0, s, order,
                           region<uint32_t>(ws, L.tiles), bs, vn);
    }
    hipLaunchKernelGGL(k_scan_blocksums, dim3(1), dim3(1024), 0, s, bs, L.nblk_vn, counters,
                       (unsigned long long)L.cap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || vn == 0) return e;
    DupArgs a;
    a.order = order;
    a.rect = region<uint2>(ws, L.rect);
    a.tiles = region<uint32_t>(ws, L.tiles);
    a.offsets = region<uint32_t>(ws, L.offsets);
    a.offk = region<uint32_t>(ws, L.offk);
    a.wstart = region<uint32_t>(ws, L.wstart);
    a.blockoff = bs;
    a.counters = counters;
    a.keys = region<uint32_t>(ws, L.keys0);
    a.vals = region<uint32_t>(ws, L.vals0);
    a.vn = vn;
    hipLaunchKernelGGL(k_offsets, dim3(L.nblk_vn), dim3(kPreprocessBlock), 0, s, a);
    hipLaunchKernelGGL(k_emit, dim3(L.nwin_max), dim3(kWindowThreads), 0, s, a, views, (int)L.n);
    return hipGetLastError();
}

}  // namespace gsp
