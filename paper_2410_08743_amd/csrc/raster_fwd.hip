// raster_fwd.hip -- per-tile instance ranges and the forward rasterizer.
//
// Sec. III-A, Eq. (3)-(4): every pixel composites, front to back in
// (depth, Gaussian index) order, the splats whose tile rectangle contains its
// tile: alpha = min(0.99, o exp(power)); splats with power > 0 or
// alpha < 1/255 are skipped; compositing stops before a splat that would
// take the transmittance below 1e-4; colour = sum c alpha T + T_final bg.
//
// MI355X design: one wavefront per 16 x 16 tile and four pixels per lane.
// The wave stages 64 list entries at a time in LDS (the list ids are read
// coalesced, the 48-byte splat records are gathered from L2/MALL) and every
// lane then reads each staged splat with a broadcast LDS load and evaluates
// it for its four pixels, so one LDS read feeds four evaluations.  A tile
// needs no barrier across waves, and the wave leaves as soon as its 256
// pixels are saturated.
#include "block_ops.h"
#include "raster_common.h"

namespace gsp {

__global__ __launch_bounds__(256) void k_ranges(const unsigned long long *keys,
                                                const uint32_t *counters, uint2 *ranges) {
    const uint32_t M = counters[kCntMEff];
    const size_t k = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= M) return;
    const uint32_t tile = (uint32_t)(keys[k] >> 32);
    if (k == 0 || (uint32_t)(keys[k - 1] >> 32) != tile) ranges[tile].x = (uint32_t)k;
    if (k == M - 1 || (uint32_t)(keys[k + 1] >> 32) != tile) ranges[tile].y = (uint32_t)(k + 1);
}

struct FwdArgs {
    const uint2 *ranges;
    const uint32_t *vals;
    const float4 *geom;
    const float4 *color;
    float *images;
    float *alphas;
    float *tfinal;
    uint32_t *ncontrib;
    uint32_t *neval;    // STATS only: entries evaluated per pixel (up to the stop)
    uint32_t *nblend;   // STATS only: entries blended per pixel
};

// STATS = true is a measurement variant that also counts, per pixel, the
// evaluated and blended (pixel, splat) pairs; the work counts define the
// kernel's algorithmic operation count.
template <bool STATS>
__global__ __launch_bounds__(kRasterThreads) void k_raster_fwd(FwdArgs a, ViewsK views) {
    __shared__ StagedSplat stage[kBatch];
    const int tile = blockIdx.x;
    const ViewK &vw = views.v[view_of_tile(views, tile)];
    const int lt = tile - vw.tile_base;
    const int tx = lt % vw.gw, ty = lt / vw.gw;
    const int px0 = vw.roi_x + kTile * tx, py0 = vw.roi_y + kTile * ty;
    const int lane = threadIdx.x;
    const int lx = lane & 15, ly = lane >> 4;
    const int rx = kTile * tx + lx;

    float T[kPixPerLane], cr[kPixPerLane], cg[kPixPerLane], cb[kPixPerLane];
    int last[kPixPerLane];
    bool live[kPixPerLane];
    uint32_t ne[kPixPerLane], nb[kPixPerLane];
#pragma unroll
    for (int q = 0; q < kPixPerLane; q++) {
        ne[q] = nb[q] = 0;
        T[q] = 1.f;
        cr[q] = cg[q] = cb[q] = 0.f;
        last[q] = 0;
        live[q] = rx < vw.roi_w && kTile * ty + ly + 4 * q < vw.roi_h;
    }
    const float fxl = (float)lx;

    const uint2 rg = a.ranges[tile];
    const int len = (int)(rg.y - rg.x);
    for (int b0 = 0; b0 < len; b0 += kBatch) {
        if (!__any(live[0] | live[1] | live[2] | live[3])) break;
        const int k = b0 + lane;
        if (k < len) {
            const uint32_t id = a.vals[rg.x + k];
            const float4 g0 = a.geom[2 * (size_t)id];
            const float4 g1 = a.geom[2 * (size_t)id + 1];
            const float4 c = a.color[id];
            StagedSplat s;
            s.a = make_float4(rel_coord(g0.x, g0.z, px0), rel_coord(g0.y, g0.w, py0), g1.x, g1.y);
            s.b = make_float4(g1.z, g1.w, c.x, c.y);
            s.c = make_float4(c.z, 0.f, 0.f, 0.f);
            stage[lane] = s;
        }
        __syncthreads();
        const int cnt = min(kBatch, len - b0);
        for (int j = 0; j < cnt; j++) {
            const float4 sa = stage[j].a;
            const float4 sb = stage[j].b;
            const float sbl = stage[j].c.x;
            const float dx = sa.x - fxl;
#pragma unroll
            for (int q = 0; q < kPixPerLane; q++) {
                const float dy = sa.y - (float)(ly + 4 * q);
                const float power = splat_power(sa.z, sa.w, sb.x, dx, dy);
                const float alpha = fminf(kAlphaMax, sb.y * __expf(power));
                const bool hit = live[q] && power <= 0.f && alpha >= kAlphaMin;
                const float testT = T[q] * (1.f - alpha);
                if (STATS && live[q]) ne[q]++;
                if (STATS && hit && testT >= kTMin) nb[q]++;
                if (hit && testT < kTMin) live[q] = false;
                if (hit && testT >= kTMin) {
                    const float wgt = alpha * T[q];
                    cr[q] = fmaf(sb.z, wgt, cr[q]);
                    cg[q] = fmaf(sb.w, wgt, cg[q]);
                    cb[q] = fmaf(sbl, wgt, cb[q]);
                    T[q] = testT;
                    last[q] = b0 + j + 1;
                }
            }
            if ((j & 7) == 7 && !__any(live[0] | live[1] | live[2] | live[3])) break;
        }
        __syncthreads();
    }

    const int P = vw.roi_w * vw.roi_h;
#pragma unroll
    for (int q = 0; q < kPixPerLane; q++) {
        const int ry = kTile * ty + ly + 4 * q;
        if (rx >= vw.roi_w || ry >= vw.roi_h) continue;
        const size_t pix = (size_t)ry * vw.roi_w + rx;
        float *img = a.images + 3 * (size_t)vw.pix_base;
        img[pix] = cr[q] + T[q] * vw.bg[0];
        img[(size_t)P + pix] = cg[q] + T[q] * vw.bg[1];
        img[2 * (size_t)P + pix] = cb[q] + T[q] * vw.bg[2];
        a.tfinal[vw.pix_base + pix] = T[q];
        a.ncontrib[vw.pix_base + pix] = (uint32_t)last[q];
        if (a.alphas) a.alphas[vw.pix_base + pix] = 1.f - T[q];
        if (STATS) {
            a.neval[vw.pix_base + pix] = ne[q];
            a.nblend[vw.pix_base + pix] = nb[q];
        }
    }
}

hipError_t launch_ranges(const Layout &L, char *ws, const uint64_t *keys, hipStream_t s) {
    uint2 *ranges = region<uint2>(ws, L.ranges);
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(ranges), 0u,
                                   2 * (int64_t)L.total_tiles, s);
    if (e != hipSuccess) return e;
    const int64_t blocks = (L.cap + 255) / 256;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<const unsigned long long *>(keys),
                       region<uint32_t>(ws, L.counters), ranges);
    return hipGetLastError();
}

hipError_t launch_raster_fwd(const ViewsK &views, const Layout &L, char *ws, const uint32_t *vals,
                             float *images, float *alphas, bool stats, hipStream_t s) {
    if (L.total_tiles == 0) return hipSuccess;
    FwdArgs a;
    a.ranges = region<uint2>(ws, L.ranges);
    a.vals = vals;
    a.geom = region<float4>(ws, L.geom);
    a.color = region<float4>(ws, L.color);
    a.images = images;
    a.alphas = alphas;
    a.tfinal = region<float>(ws, L.tfinal);
    a.ncontrib = region<uint32_t>(ws, L.ncontrib);
    a.neval = region<uint32_t>(ws, L.stats);
    a.nblend = a.neval + L.total_pix;
    if (stats)
        hipLaunchKernelGGL(k_raster_fwd<true>, dim3(L.total_tiles), dim3(kRasterThreads), 0, s, a, views);
    else
        hipLaunchKernelGGL(k_raster_fwd<false>, dim3(L.total_tiles), dim3(kRasterThreads), 0, s, a, views);
    return hipGetLastError();
}

}  // namespace gsp
