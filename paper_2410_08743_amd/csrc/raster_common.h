// raster_common.h -- per-pixel splat evaluation shared by the forward and
// backward rasterizers, so that the backward's recomputation takes exactly
// the forward's decisions (same operations in the same order).
//
// Sec. III-A, Eq. (3): alpha = o exp(-1/2 d^T Sigma_hat^-1 d), d = pixel -
// mu_hat, with Sigma_hat^-1 = [[A, B], [B, C]] (the paper prints Sigma_hat
// where its inverse is meant).
#pragma once

#include <hip/hip_runtime.h>

#include "gsp_internal.h"

namespace gsp {

// One wavefront (64 lanes) rasterizes one 16 x 16 tile; lane l owns pixels
// (l % 16, l / 16 + 4 q) for q = 0..3.
constexpr int kRasterThreads = 64;
constexpr int kPixPerLane = 4;
constexpr int kBatch = 64;          // list entries staged in LDS at a time

// Splat as staged in LDS: centre relative to the tile's first pixel, conic,
// opacity, colour and (backward only) the instance's slot index.
struct StagedSplat {
    float4 a;   // u_rel, v_rel, A, B
    float4 b;   // C, o, r, g
    float4 c;   // b, slot (bits), 0, 0
};

__device__ __forceinline__ float splat_power(float A, float B, float C, float dx, float dy) {
#pragma clang fp contract(off)
    const float q = __fmaf_rn(A * dx, dx, (C * dy) * dy);
    return __fmaf_rn(-0.5f, q, -((B * dx) * dy));
}

// Centre of a splat relative to pixel (px0, py0), from its (hi, lo) pair.
__device__ __forceinline__ float rel_coord(float hi, float lo, int origin) {
#pragma clang fp contract(off)
    return (hi - (float)origin) + lo;
}

__device__ __forceinline__ int view_of_tile(const ViewsK &views, int tile) {
    int v = 0;
    while (v + 1 < views.count && tile >= views.v[v + 1].tile_base) v++;
    return v;
}

}  // namespace gsp
