// raster_common.h -- per-pixel splat evaluation shared by the forward and
// backward rasterizers, so that the backward's recomputation takes exactly
// the forward's decisions (same operations in the same order).
//
// Sec. III-A, Eq. (3): alpha = o exp(power), power = -1/2 d^T Sigma_hat^-1 d
// with d = pixel - mu_hat and Sigma_hat^-1 = [[A, B], [B, C]] (the paper
// prints Sigma_hat where its inverse is meant), so
// power = -1/2 (A dx^2 + C dy^2) - B dx dy.
//
// The preprocess stores the conic pre-scaled to base 2,
// (A2, B2, C2) = -log2(e) (A/2, B, C/2), and lo = log2(o), so that
// p2 = log2(e) power = A2 dx^2 + B2 dx dy + C2 dy^2 and alpha = 2^(p2 + lo):
// two FMAs and one v_exp_f32 per pixel once the dx terms, which the pixels
// of a lane share (they lie in one column), are formed.
#pragma once

#include <hip/hip_runtime.h>

#include "gsp_internal.h"

namespace gsp {

// SPLIT wavefronts (64 lanes each) rasterize one 16 x 16 tile, each a
// horizontal strip of 16 / SPLIT rows; in part h, lane l owns pixels
// (l % 16, 16 h / SPLIT + l / 16 + 4 q) for q < 4 / SPLIT, so the q-th
// pixels of all lanes form the 16 x 4 band 4 h / SPLIT + q of the tile.
// The parts of a tile are independent workgroups: more of them keep the
// SIMDs busy (a 1008 x 756 view has only 3024 tiles) and each walks, culls
// and stops for its own rows.
constexpr int kRasterThreads = 64;
constexpr int kBatch = 64;          // list entries staged in LDS at a time
static_assert(kChunk % kBatch == 0, "the backward's chunks start at batch boundaries");
#ifndef GSP_FWD_UNROLL
#define GSP_FWD_UNROLL 2
#endif
constexpr int kUnroll = GSP_FWD_UNROLL;   // entries per step of the inner loop

constexpr float kLn2 = 0.6931471805599453f;
// A splat can reach alpha >= 1/255 at a pixel only if p2 + log2(o) is at least
// log2(1/255); the 0.01 margin keeps the test (taken as p2 >= this - log2(o))
// conservative with respect to v_exp_f32's and the subtraction's rounding, so
// skipping on it never changes a decision.
constexpr float kLog2AlphaMinLoose = -7.994353436858858f - 0.01f;
// log2 of an opacity that keeps every unclamped alpha of its splat below the
// 0.99 clamp: exp2(-0.0155) = 0.98931, so with power <= 0 the alpha stays
// below 0.99 by far more than the error of the exp2 instruction, and
// min(0.99, alpha) is alpha itself.
constexpr float kLoNoClamp = -0.0155f;

// Splat as staged in LDS: centre relative to the tile's first pixel, scaled
// conic, log2 opacity and colour; the forward adds its list position + 1, the
// backward its list position, the instance's slot and 1/o.  Every lane reads
// every staged byte, so the forward's record is kept to 40 bytes.
struct StagedA { float u, v, A2, B2; };
struct StagedB { float C2, lo, r, g; };
struct StagedF { float b; uint32_t jp1; };
struct StagedC { float b, inv_o; uint32_t slot, pm; };   // pm: list position

// Row offset that marks a pixel as done: every splat's p2 there is -inf, so
// the candidate test (p2 >= lim) fails without a separate flag.
constexpr float kInactiveRow = 1e30f;

// Centre of a splat relative to pixel (px0, py0), from its (hi, lo) pair.
__device__ __forceinline__ float rel_coord(float hi, float lo, int origin) {
#pragma clang fp contract(off)
    return (hi - (float)origin) + lo;
}

// Per (lane, splat) terms shared by the pixels of a lane (one column).
struct ColTerms {
    float dx, adx2, bdx;
};

__device__ __forceinline__ ColTerms col_terms(const StagedA &s, float px) {
#pragma clang fp contract(off)
    ColTerms t;
    t.dx = s.u - px;
    t.adx2 = (s.A2 * t.dx) * t.dx;
    t.bdx = s.B2 * t.dx;
    return t;
}

// log2(e) * power at a pixel with offset dy.
__device__ __forceinline__ float splat_p2(const ColTerms &t, float C2, float dy) {
#pragma clang fp contract(off)
    return __fmaf_rn(dy, __fmaf_rn(C2, dy, t.bdx), t.adx2);
}

// Pre-clamp opacity o * exp(power).
__device__ __forceinline__ float splat_alpha_pre(float p2, float lo) {
#pragma clang fp contract(off)
    return __builtin_amdgcn_exp2f(p2 + lo);
}

// Bit q of the result is set when some pixel of rows row0 + 4q .. row0 + 4q + 3
// of the tile (q < 4 / SPLIT) may reach alpha >= 1/255, i.e. when the rasterizer's own candidate test
// (p2 >= kLog2AlphaMinLoose - lo) may pass there; a clear bit is a proof that
// it fails at every pixel of those rows.  Per pixel row, p2 is a concave
// quadratic in dx whose maximum over the row's dx range [u - 15, u] is taken
// at the clamped stationary point.  The margin covers the float32 rounding of
// both this bound and the rasterizer's evaluation: 0.02 plus 1e-5 times the
// largest magnitude the three terms of p2 take in the row, some forty times
// the error of either three-operation evaluation.
template <int SPLIT>
__device__ __forceinline__ uint32_t band_mask(float u, float v, float A2, float B2, float C2,
                                              float lo, int row0) {
    constexpr int kRows = kTile / SPLIT;
    if (!(A2 < 0.f) || !(C2 < 0.f)) return (1u << (4 / SPLIT)) - 1u;   // not negative definite
    const float xa = u - (float)(kTile - 1), xb = u;
    const float dxm = fmaxf(fabsf(xa), fabsf(xb));
    const float half_inv = -0.5f / A2;
    const float thr = kLog2AlphaMinLoose - lo;
    const float adxm2 = fabsf(A2) * dxm * dxm;
    uint32_t mask = 0u;
#pragma unroll
    for (int r = 0; r < kRows; r++) {
        const float dy = v - (float)(row0 + r);
        const float bdy = B2 * dy;
        const float cdy2 = C2 * dy * dy;
        const float xs = fminf(fmaxf(bdy * half_inv, xa), xb);
        const float m = fmaf(fmaf(A2, xs, bdy), xs, cdy2);
        const float mag = adxm2 + fabsf(bdy) * dxm + fabsf(cdy2);
        if (m + fmaf(1e-5f, mag, 0.02f) >= thr) mask |= 1u << (r >> 2);
    }
    return mask;
}

// Position of a lane's entry among the entries of its wavefront that are
// kept, counting lanes below it.
__device__ __forceinline__ int kept_rank(unsigned long long kept) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(kept >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)kept, 0u));
}

// Workgroup -> (rank of the tile in launch order, part).  The SPLIT parts
// of one tile go to workgroups 8 apart, which the dispatcher places on the
// same XCD (workgroups are dealt round-robin over the 8 XCDs), so the later
// parts find the tile's splat records in that XCD's L2.
template <int SPLIT>
__device__ __forceinline__ void part_of_block(int b, int &rank, int &part) {
    if (SPLIT == 1) {
        rank = b;
        part = 0;
    } else {
        const int grp = b / (8 * SPLIT), r = b % (8 * SPLIT);
        rank = grp * 8 + (r & 7);
        part = r >> 3;
    }
}

// Workgroups of a rasterizer launch over `tiles` tiles (a multiple of
// 8 SPLIT when split; the extra ones exit at once).
template <int SPLIT>
inline int raster_blocks(int tiles) {
    return SPLIT == 1 ? tiles : ((tiles + 7) / 8) * 8 * SPLIT;
}

__device__ __forceinline__ int view_of_tile(const ViewsK &views, int tile) {
    int v = 0;
    while (v + 1 < views.count && tile >= views.v[v + 1].tile_base) v++;
    return v;
}

}  // namespace gsp
