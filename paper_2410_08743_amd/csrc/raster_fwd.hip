// raster_fwd.hip -- per-tile instance ranges and the forward rasterizer.
//
// Sec. III-A, Eq. (3)-(4): every pixel composites, front to back in
// (depth, Gaussian index) order, the splats whose tile rectangle contains its
// tile: alpha = min(0.99, o exp(power)); splats with power > 0 or
// alpha < 1/255 are skipped; compositing stops before a splat that would
// take the transmittance below 1e-4; colour = sum c alpha T + T_final bg.
//
// MI355X design: one wavefront per 16 x 16 tile and four pixels per lane, the
// four in one column so that they share the splat's dx terms.  The wave
// stages 64 list entries at a time in LDS (list ids read coalesced, splat
// records gathered from L2/MALL; entries past the end are inert), and the
// inner loop runs eight entries per step without bounds checks, each entry a
// broadcast LDS read that feeds four pixel evaluations of two FMAs and one
// v_exp_f32.  A tile needs no barrier across waves, and the wave leaves as
// soon as its 256 pixels are saturated.
#include "block_ops.h"
#include "raster_common.h"

namespace gsp {

__global__ __launch_bounds__(256) void k_ranges(const uint32_t *keys, const uint32_t *counters,
                                                uint2 *ranges) {
    const uint32_t M = counters[kCntMEff];
    const size_t k = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= M) return;
    const uint32_t tile = keys[k];
    if (k == 0 || keys[k - 1] != tile) ranges[tile].x = (uint32_t)k;
    if (k == M - 1 || keys[k + 1] != tile) ranges[tile].y = (uint32_t)(k + 1);
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
    __shared__ StagedA sA[kBatch];
    __shared__ StagedB sB[kBatch];
    __shared__ float sCb[kBatch];
    const int tile = blockIdx.x;
    const ViewK &vw = views.v[view_of_tile(views, tile)];
    const int lt = tile - vw.tile_base;
    const int tx = lt % vw.gw, ty = lt / vw.gw;
    const int px0 = vw.roi_x + kTile * tx, py0 = vw.roi_y + kTile * ty;
    const int lane = threadIdx.x;
    const int lx = lane & 15, ly = lane >> 4;
    const int rx = kTile * tx + lx;

    // T > 0 while a pixel composites; a pixel that stopped (or lies outside
    // the region) keeps -T, so later splats can neither blend nor restart it.
    float T[kPixPerLane], cr[kPixPerLane], cg[kPixPerLane], cb[kPixPerLane], fy[kPixPerLane];
    int last[kPixPerLane];
    uint32_t ne[kPixPerLane], nb[kPixPerLane];
#pragma unroll
    for (int q = 0; q < kPixPerLane; q++) {
        ne[q] = nb[q] = 0;
        const bool in = rx < vw.roi_w && kTile * ty + ly + 4 * q < vw.roi_h;
        T[q] = in ? 1.f : -1.f;
        cr[q] = cg[q] = cb[q] = 0.f;
        last[q] = 0;
        fy[q] = (float)(ly + 4 * q);
    }
    const float fxl = (float)lx;

    const uint2 rg = a.ranges[tile];
    const int len = (int)(rg.y - rg.x);

    // records of the batch being staged, gathered one batch ahead
    float4 g0 = make_float4(0.f, 0.f, 0.f, 0.f), g1 = make_float4(0.f, 0.f, 0.f, -INFINITY),
           gc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (lane < len) {
        const uint32_t id = a.vals[rg.x + lane];
        g0 = a.geom[2 * (size_t)id];
        g1 = a.geom[2 * (size_t)id + 1];
        gc = a.color[id];
    }
    for (int b0 = 0; b0 < len; b0 += kBatch) {
        if (!__any(T[0] > 0.f || T[1] > 0.f || T[2] > 0.f || T[3] > 0.f)) break;
        sA[lane] = StagedA{rel_coord(g0.x, g0.z, px0), rel_coord(g0.y, g0.w, py0), g1.x, g1.y};
        sB[lane] = StagedB{g1.z, g1.w, gc.x, gc.y};
        sCb[lane] = gc.z;
        __syncthreads();
        {
            const int k = b0 + kBatch + lane;
            g0 = make_float4(0.f, 0.f, 0.f, 0.f);
            g1 = make_float4(0.f, 0.f, 0.f, -INFINITY);   // inert: alpha = 0
            gc = make_float4(0.f, 0.f, 0.f, 0.f);
            if (k < len) {
                const uint32_t id = a.vals[rg.x + k];
                g0 = a.geom[2 * (size_t)id];
                g1 = a.geom[2 * (size_t)id + 1];
                gc = a.color[id];
            }
        }
        for (int j0 = 0; j0 < kBatch; j0 += kUnroll) {
            StagedA es[kUnroll];
            StagedB et[kUnroll];
            float eb[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; u++) {
                es[u] = sA[j0 + u];
                et[u] = sB[j0 + u];
                eb[u] = sCb[j0 + u];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; u++) {
                const int j = b0 + j0 + u;
                const ColTerms ct = col_terms(es[u], fxl);
                float p2[kPixPerLane];
                bool cand = false;
#pragma unroll
                for (int q = 0; q < kPixPerLane; q++) {
                    p2[q] = splat_p2(ct, et[u].C2, es[u].v - fy[q]);
                    cand |= T[q] > 0.f && p2[q] <= 0.f && p2[q] + et[u].lo >= kLog2AlphaMinLoose;
                }
                if (STATS) {
#pragma unroll
                    for (int q = 0; q < kPixPerLane; q++)
                        if (T[q] > 0.f && j < len) ne[q]++;
                }
                // no pixel of the tile can reach 1/255: nothing to do
                if (!__any(cand)) continue;
#pragma unroll
                for (int q = 0; q < kPixPerLane; q++) {
                    const float alpha = fminf(kAlphaMax, splat_alpha_pre(p2[q], et[u].lo));
                    const float testT = T[q] * (1.f - alpha);
                    const bool hit = p2[q] <= 0.f && alpha >= kAlphaMin;
                    const bool blend = hit && testT >= kTMin;
                    const bool stop = hit && testT < kTMin;
                    if (STATS && blend) nb[q]++;
                    const float wgt = blend ? alpha * T[q] : 0.f;
                    cr[q] = fmaf(et[u].r, wgt, cr[q]);
                    cg[q] = fmaf(et[u].g, wgt, cg[q]);
                    cb[q] = fmaf(eb[u], wgt, cb[q]);
                    last[q] = blend ? j + 1 : last[q];
                    T[q] = blend ? testT : (stop ? -fabsf(T[q]) : T[q]);
                }
            }
            if (!__any(T[0] > 0.f || T[1] > 0.f || T[2] > 0.f || T[3] > 0.f) ||
                b0 + j0 + kUnroll >= len)
                break;
        }
        __syncthreads();
    }

    const int P = vw.roi_w * vw.roi_h;
#pragma unroll
    for (int q = 0; q < kPixPerLane; q++) {
        const int ry = kTile * ty + ly + 4 * q;
        if (rx >= vw.roi_w || ry >= vw.roi_h) continue;
        const size_t pix = (size_t)ry * vw.roi_w + rx;
        const float Tf = fabsf(T[q]);
        float *img = a.images + 3 * (size_t)vw.pix_base;
        img[pix] = cr[q] + Tf * vw.bg[0];
        img[(size_t)P + pix] = cg[q] + Tf * vw.bg[1];
        img[2 * (size_t)P + pix] = cb[q] + Tf * vw.bg[2];
        a.tfinal[vw.pix_base + pix] = Tf;
        a.ncontrib[vw.pix_base + pix] = (uint32_t)last[q];
        if (a.alphas) a.alphas[vw.pix_base + pix] = 1.f - Tf;
        if (STATS) {
            a.neval[vw.pix_base + pix] = ne[q];
            a.nblend[vw.pix_base + pix] = nb[q];
        }
    }
}

hipError_t launch_ranges(const Layout &L, char *ws, const uint32_t *keys, hipStream_t s) {
    uint2 *ranges = region<uint2>(ws, L.ranges);
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(ranges), 0u,
                                   2 * (int64_t)L.total_tiles, s);
    if (e != hipSuccess) return e;
    const int64_t blocks = (L.cap + 255) / 256;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)blocks), dim3(256), 0, s, keys,
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
