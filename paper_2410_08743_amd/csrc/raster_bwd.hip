// raster_bwd.hip -- backward of the compositing of Eq. (3)-(4).
//
// For the blended entries i of a pixel, with upstream G = dL/dC and T_i the
// transmittance in front of i:
//   dL/dc_i     = G alpha_i T_i
//   dL/dalpha_i = T_i G . (c_i - S_i),  S_i = colour behind i seen through i,
//   S_last = bg,  S_{i-1} = alpha_i c_i + (1 - alpha_i) S_i
// and through alpha = o exp(power) (no gradient when clamped at 0.99) to the
// opacity, the conic and the projected centre.
//
// MI355X design: nothing per pixel is stored by the forward beyond T_final
// and the contributor count; each wavefront walks its tile's list back to
// front from the largest contributor count, recovering T_i = T_{i+1} /
// (1 - alpha_i) with the forward's exact arithmetic.  The four pixels of a
// lane are summed in registers and the 64 lanes with a butterfly of
// cross-lane adds, giving one 9-float partial per (tile, splat) that is
// written to the instance's own slot (its position in emission order).  No
// atomics: the per-splat reduction over its slots happens later in a fixed
// order, so gradients are bit-reproducible.
#include "block_ops.h"
#include "raster_common.h"

namespace gsp {

struct BwdArgs {
    const uint2 *ranges;
    const uint32_t *vals;
    const float4 *geom;
    const float4 *color;
    const uint2 *rect;
    const uint32_t *offsets;
    const float *dl;
    const float *tfinal;
    const uint32_t *ncontrib;
    float *slots;          // [9][cap]
    size_t cap;
};

// Slot of the instance of splat `id` in tile (tx, ty): its emission position.
__device__ __forceinline__ uint32_t slot_of(const BwdArgs &a, uint32_t id, int tx, int ty) {
    const uint2 r = a.rect[id];
    const int x0 = r.x & 0xffff, y0 = r.x >> 16, x1 = r.y & 0xffff;
    return a.offsets[id] + (uint32_t)((ty - y0) * (x1 - x0) + (tx - x0));
}

__global__ __launch_bounds__(kRasterThreads) void k_raster_bwd(BwdArgs a, ViewsK views) {
    __shared__ StagedSplat stage[kBatch];
    const int tile = blockIdx.x;
    const ViewK &vw = views.v[view_of_tile(views, tile)];
    const int lt = tile - vw.tile_base;
    const int tx = lt % vw.gw, ty = lt / vw.gw;
    const int px0 = vw.roi_x + kTile * tx, py0 = vw.roi_y + kTile * ty;
    const int lane = threadIdx.x;
    const int lx = lane & 15, ly = lane >> 4;
    const int rx = kTile * tx + lx;
    const int P = vw.roi_w * vw.roi_h;

    float T[kPixPerLane], G[kPixPerLane][3], S[kPixPerLane][3];
    int last[kPixPerLane];
    int maxlast = 0;
#pragma unroll
    for (int q = 0; q < kPixPerLane; q++) {
        const int ry = kTile * ty + ly + 4 * q;
        const bool in = rx < vw.roi_w && ry < vw.roi_h;
        const size_t pix = (size_t)ry * vw.roi_w + rx;
        T[q] = in ? a.tfinal[vw.pix_base + pix] : 1.f;
        last[q] = in ? (int)a.ncontrib[vw.pix_base + pix] : 0;
        const float *dl = a.dl + 3 * (size_t)vw.pix_base;
        G[q][0] = in ? dl[pix] : 0.f;
        G[q][1] = in ? dl[(size_t)P + pix] : 0.f;
        G[q][2] = in ? dl[2 * (size_t)P + pix] : 0.f;
        S[q][0] = vw.bg[0];
        S[q][1] = vw.bg[1];
        S[q][2] = vw.bg[2];
        maxlast = max(maxlast, last[q]);
    }
    maxlast = wave_max(maxlast);
    const float fxl = (float)lx;

    const uint2 rg = a.ranges[tile];
    const int len = (int)(rg.y - rg.x);
    // entries no pixel blended get zero slots
    for (int k = maxlast + lane; k < len; k += kBatch) {
        const uint32_t e = slot_of(a, a.vals[rg.x + k], tx, ty);
#pragma unroll
        for (int c = 0; c < 9; c++) a.slots[c * a.cap + e] = 0.f;
    }

    for (int hi = maxlast; hi > 0; hi -= kBatch) {
        const int lo = max(0, hi - kBatch);
        const int k = lo + lane;
        if (k < hi) {
            const uint32_t id = a.vals[rg.x + k];
            const float4 g0 = a.geom[2 * (size_t)id];
            const float4 g1 = a.geom[2 * (size_t)id + 1];
            const float4 c = a.color[id];
            StagedSplat s;
            s.a = make_float4(rel_coord(g0.x, g0.z, px0), rel_coord(g0.y, g0.w, py0), g1.x, g1.y);
            s.b = make_float4(g1.z, g1.w, c.x, c.y);
            s.c = make_float4(c.z, __uint_as_float(slot_of(a, id, tx, ty)), 0.f, 0.f);
            stage[lane] = s;
        }
        __syncthreads();
        for (int j = hi - lo - 1; j >= 0; j--) {
            const int pos = lo + j;
            const float4 sa = stage[j].a;
            const float4 sb = stage[j].b;
            const float4 sc = stage[j].c;
            const float dx = sa.x - fxl;
            const float col[3] = {sb.z, sb.w, sc.x};
            float acc[9];
#pragma unroll
            for (int c = 0; c < 9; c++) acc[c] = 0.f;
#pragma unroll
            for (int q = 0; q < kPixPerLane; q++) {
                const float dy = sa.y - (float)(ly + 4 * q);
                const float power = splat_power(sa.z, sa.w, sb.x, dx, dy);
                const float ex = __expf(power);
                const float apre = sb.y * ex;
                const float alpha = fminf(kAlphaMax, apre);
                if (pos < last[q] && power <= 0.f && alpha >= kAlphaMin) {
                    T[q] = T[q] / (1.f - alpha);
                    const float wgt = alpha * T[q];
                    float dalpha = 0.f;
#pragma unroll
                    for (int ch = 0; ch < 3; ch++) {
                        acc[6 + ch] = fmaf(G[q][ch], wgt, acc[6 + ch]);
                        dalpha = fmaf(G[q][ch], col[ch] - S[q][ch], dalpha);
                        S[q][ch] = fmaf(alpha, col[ch] - S[q][ch], S[q][ch]);
                    }
                    dalpha *= T[q];
                    if (apre <= kAlphaMax) {
                        acc[5] = fmaf(dalpha, ex, acc[5]);
                        const float dp = dalpha * alpha;
                        acc[0] -= dp * fmaf(sa.z, dx, sa.w * dy);
                        acc[1] -= dp * fmaf(sb.x, dy, sa.w * dx);
                        acc[2] -= 0.5f * dp * dx * dx;
                        acc[3] -= dp * dx * dy;
                        acc[4] -= 0.5f * dp * dy * dy;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < 9; c++) acc[c] = wave_sum(acc[c]);
            if (lane == 0) {
                const uint32_t e = __float_as_uint(sc.y);
#pragma unroll
                for (int c = 0; c < 9; c++) a.slots[c * a.cap + e] = acc[c];
            }
        }
        __syncthreads();
    }
}

hipError_t launch_raster_bwd(const ViewsK &views, const Layout &L, char *ws, const uint32_t *vals,
                             const float *dl_dimages, hipStream_t s) {
    if (L.total_tiles == 0) return hipSuccess;
    BwdArgs a;
    a.ranges = region<uint2>(ws, L.ranges);
    a.vals = vals;
    a.geom = region<float4>(ws, L.geom);
    a.color = region<float4>(ws, L.color);
    a.rect = region<uint2>(ws, L.rect);
    a.offsets = region<uint32_t>(ws, L.offsets);
    a.dl = dl_dimages;
    a.tfinal = region<float>(ws, L.tfinal);
    a.ncontrib = region<uint32_t>(ws, L.ncontrib);
    a.slots = region<float>(ws, L.slots);
    a.cap = (size_t)L.cap;
    hipLaunchKernelGGL(k_raster_bwd, dim3(L.total_tiles), dim3(kRasterThreads), 0, s, a, views);
    return hipGetLastError();
}

}  // namespace gsp
