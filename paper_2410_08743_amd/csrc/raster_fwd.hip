// raster_fwd.hip -- per-tile instance ranges and the forward rasterizer.
//
// Sec. III-A, Eq. (3)-(4): every pixel composites, front to back in
// (depth, Gaussian index) order, the splats whose tile rectangle contains its
// tile: alpha = min(0.99, o exp(power)); splats with power > 0 or
// alpha < 1/255 are skipped; compositing stops before a splat that would
// take the transmittance below 1e-4; colour = sum c alpha T + T_final bg.
//
// MI355X design: kSplit wavefronts per 16 x 16 tile, each a strip of rows
// with the pixels of a lane in one column so that they share the splat's dx
// terms.  A wave stages 64 list entries at a time in LDS (list ids read
// coalesced, splat records gathered one batch ahead), keeping only the
// entries that can reach 1/255 in its rows (each lane bounds its own entry,
// then a ballot compacts the batch), and its inner loop runs the kept
// entries a few at a time, each a broadcast LDS read that feeds the lane's
// pixel evaluations of two FMAs and one v_exp_f32.  The waves of a tile need
// no barrier between them, and each leaves as soon as its pixels are
// saturated.
#include <type_traits>

#include "block_ops.h"
#include "raster_common.h"

namespace gsp {

constexpr int kSplit = kSplitFwd;
constexpr int kPixPerLane = 4 / kSplit;   // pixels per lane, one column

__global__ __launch_bounds__(256) void k_ranges(const uint32_t *keys, const uint32_t *counters,
                                                uint2 *ranges) {
    const uint32_t M = counters[kCntMEff];
    const size_t k = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= M) return;
    const uint32_t tile = keys[k];
    if (k == 0 || keys[k - 1] != tile) ranges[tile].x = (uint32_t)k;
    if (k == M - 1 || keys[k + 1] != tile) ranges[tile].y = (uint32_t)(k + 1);
}

// Launch order of the tiles: longest lists first (in buckets of 4 entries:
// 256 buckets spread the same-address LDS atomics of the counting sort
// four times thinner than buckets of 16), so that the longest tiles do not
// start last and leave a tail.
// The same kernel lists the backward work items (tile, chunk), also longest
// first by chunk length; their count goes to counters[kCntItems].  The
// orders only decide which workgroup takes which tile or chunk; every
// result is the same in any order.
constexpr int kOrderBuckets = 256;
constexpr int kOrderThreads = 1024;
constexpr int kOrderRounds = 8;   // tiles per thread whose ranges are loaded together

__host__ __device__ constexpr int order_bucket(int len) {
    return kOrderBuckets - 1 - ((len >> 2) < kOrderBuckets - 1 ? (len >> 2) : kOrderBuckets - 1);
}

__global__ __launch_bounds__(kOrderThreads) void k_tile_order(const uint2 *ranges, int total_tiles,
                                                             uint32_t *order, uint32_t *items,
                                                             uint32_t *counters) {
    // Full chunks all fall into one bucket; a wave adds its tiles' full
    // chunks there with one atomic (same-address LDS atomics serialise).
    constexpr int kFull = order_bucket(kChunk);
    __shared__ uint32_t cnt[2][kOrderBuckets], base[2][kOrderBuckets];
    const int t = threadIdx.x, lane = t & (kWave - 1);
    if (t < kOrderBuckets) cnt[0][t] = cnt[1][t] = 0;
    __syncthreads();
    constexpr int kStep = kOrderThreads * kOrderRounds;
    // lengths of this thread's tiles in the group starting at k0 (-1 past the last tile)
    auto load = [&](int k0, int (&len)[kOrderRounds]) {
#pragma unroll
        for (int r = 0; r < kOrderRounds; r++) {
            const int k = k0 + r * kOrderThreads + t;
            const uint2 rg = k < total_tiles ? ranges[k] : make_uint2(1u, 0u);
            len[r] = (int)(rg.y - rg.x);
        }
    };
    const int wave0 = t - lane;   // first thread of this wave
    // the first group's lengths serve both passes (a call with at most kStep
    // tiles loads its ranges once)
    int len_first[kOrderRounds];
    load(0, len_first);
    for (int k0 = 0; k0 < total_tiles; k0 += kStep) {
        int len[kOrderRounds];
        if (k0 == 0) {
#pragma unroll
            for (int r = 0; r < kOrderRounds; r++) len[r] = len_first[r];
        } else {
            load(k0, len);
        }
        uint32_t full = 0;   // this thread's full chunks in the round
#pragma unroll
        for (int r = 0; r < kOrderRounds; r++) {
            if (k0 + r * kOrderThreads + wave0 >= total_tiles) break;   // whole wave past the end
            if (len[r] < 0) continue;
            const int nch = chunks_of(len[r]);
            atomicAdd(&cnt[0][order_bucket(len[r])], 1u);
            atomicAdd(&cnt[1][order_bucket(len[r] - (nch - 1) * kChunk)], 1u);
            full += (uint32_t)(nch - 1);
        }
        const uint32_t wfull = wave_sum(full);
        if (lane == 0 && wfull > 0) atomicAdd(&cnt[1][kFull], wfull);
    }
    __syncthreads();
    // exclusive scans of the two bucket histograms: one wave, a bucket per lane
    static_assert(kOrderBuckets == 4 * kWave, "four buckets per lane");
    if (t < kWave) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
            uint32_t c[4], s = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                c[j] = cnt[h][4 * lane + j];
                s += c[j];
            }
            const uint32_t inc = wave_inclusive_scan(s);
            uint32_t e = inc - s;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                base[h][4 * lane + j] = e;
                e += c[j];
            }
            if (h == 1 && lane == kWave - 1) counters[kCntItems] = inc;
        }
    }
    __syncthreads();
    for (int k0 = 0; k0 < total_tiles; k0 += kStep) {
        int len[kOrderRounds];
        if (k0 == 0) {
#pragma unroll
            for (int r = 0; r < kOrderRounds; r++) len[r] = len_first[r];
        } else {
            load(k0, len);
        }
        uint32_t full = 0;
#pragma unroll
        for (int r = 0; r < kOrderRounds; r++) full += len[r] >= 0 ? (uint32_t)(chunks_of(len[r]) - 1) : 0u;
        const uint32_t wfull = wave_sum(full);
        uint32_t wb = 0;
        if (lane == 0 && wfull > 0) wb = atomicAdd(&base[1][kFull], wfull);
        wb = __shfl(wb, 0, kWave);   // the wave's first full-chunk item
        const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
        for (int r = 0; r < kOrderRounds; r++) {
            if (k0 + r * kOrderThreads + wave0 >= total_tiles) break;
            const uint32_t k = (uint32_t)(k0 + r * kOrderThreads + t);
            const int nch = len[r] >= 0 ? chunks_of(len[r]) : 1;
            if (len[r] >= 0) {
                order[atomicAdd(&base[0][order_bucket(len[r])], 1u)] = k;
                items[atomicAdd(&base[1][order_bucket(len[r] - (nch - 1) * kChunk)], 1u)] =
                    k * kMaxChunks + (uint32_t)(nch - 1);
            }
            // full chunks j of the wave's tiles, compacted by ballot so that
            // each store covers consecutive items
            for (int j = 0; j < kMaxChunks - 1; j++) {
                const unsigned long long m = __ballot(j < nch - 1);
                if (m == 0ull) break;
                if (j < nch - 1) items[wb + (uint32_t)__popcll(m & below)] = k * kMaxChunks + (uint32_t)j;
                wb += (uint32_t)__popcll(m);
            }
        }
    }
}

struct FwdArgs {
    const uint32_t *order;
    const uint2 *ranges;
    const uint32_t *vals;
    const float4 *geom;
    const float4 *color;
    float *tfinal;
    uint32_t *ncontrib;
    uint32_t *neval;    // STATS only: entries evaluated per pixel (up to the stop)
    uint32_t *nblend;   // STATS only: entries blended per pixel
    float4 *ckpt;       // per cut and tile pixel: (T, colour in front of the cut)
    float *cfinal;      // [3][total_pix]: final colour, for tiles with cuts
    // L1-fused forward: each view's img holds dL/dimage of the mean absolute
    // error against the target its dl points to (instead of the image), and
    // with l1part each wave leaves its FP64 sum of |image - target| at
    // [tile * kSplit + part]
    double *l1part;
    int total_pix;
    int total_tiles;
    bool l1;
};

template <int N>
__device__ __forceinline__ bool any_active(const float (&fy)[N]) {
    bool a = false;
#pragma unroll
    for (int q = 0; q < N; q++) a |= fy[q] != kInactiveRow;
    return wave_any(a);
}

// STATS = true is a measurement variant that also counts, per pixel, the
// evaluated and blended (pixel, splat) pairs of the algorithm -- every list
// entry up to the pixel's stop counts as evaluated, culled or not; the work
// counts define the kernel's algorithmic operation count.
template <bool STATS>
__global__ __launch_bounds__(kRasterThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_raster_fwd(FwdArgs a, ViewsK views) {
    __shared__ StagedA sA[kBatch];
    __shared__ StagedB sB[kBatch];
    __shared__ StagedF sF[kBatch];
    int rank, part;
    part_of_block<kSplit>(blockIdx.x, rank, part);
    if (rank >= a.total_tiles) return;
    const int tile = (int)a.order[rank];
    const ViewK &vw = views.v[view_of_tile(views, tile)];
    const int lt = tile - vw.tile_base;
    const int tx = lt % vw.gw, ty = lt / vw.gw;
    const int px0 = vw.roi_x + kTile * tx, py0 = vw.roi_y + kTile * ty;
    const int lane = threadIdx.x;
    const int lx = lane & 15, ly = lane >> 4;
    const int rx = kTile * tx + lx;
    const int row0 = part * (kTile / kSplit);   // first tile row of this part

    // A pixel composites while its row offset fy is finite; one that stopped
    // (or lies outside the region) gets kInactiveRow, so that no later splat
    // is a candidate there.
    float T[kPixPerLane], cr[kPixPerLane], cg[kPixPerLane], cb[kPixPerLane], fy[kPixPerLane];
    int last[kPixPerLane];
    uint32_t ne[kPixPerLane], nb[kPixPerLane];
#pragma unroll
    for (int q = 0; q < kPixPerLane; q++) {
        ne[q] = nb[q] = 0;
        const int ryl = row0 + ly + 4 * q;
        const bool in = rx < vw.roi_w && kTile * ty + ryl < vw.roi_h;
        T[q] = 1.f;
        cr[q] = cg[q] = cb[q] = 0.f;
        last[q] = 0;
        fy[q] = in ? (float)ryl : kInactiveRow;
    }
    const float fxl = (float)lx;

    const uint2 rg = a.ranges[tile];
    const int len = (int)(rg.y - rg.x);

    // records of the batch being staged, gathered one batch ahead
    float4 g0, g1, gc;
    auto gather = [&](int k) {
        g0 = make_float4(0.f, 0.f, 0.f, 0.f);
        g1 = make_float4(-1.f, 0.f, -1.f, -INFINITY);   // inert: alpha = 0
        gc = make_float4(0.f, 0.f, 0.f, 0.f);
        if (k < len) {
            const uint32_t id = a.vals[rg.x + k];
            g0 = a.geom[2 * (size_t)id];
            g1 = a.geom[2 * (size_t)id + 1];
            gc = a.color[id];
        }
    };
    // Cuts of the list for the backward's chunks (at multiples of kChunk):
    // at each cut the transmittance and accumulated colour of the pixels
    // still compositing are recorded, and the pixels that blend past the
    // first cut also store their final colour; the backward reads them only
    // for pixels that blend past the cut that ends its chunk.
    const int ncut = chunks_of(len) - 1;
    int cuts_done = 0;
    gather(lane);
    for (int b0 = 0; b0 < len; b0 += kBatch) {
        if (!any_active(fy)) break;
        if (cuts_done < ncut && b0 == (cuts_done + 1) * kChunk) {
            // The lane index is read here, not reused from the kernel's
            // start, so that no per-lane record address stays live through
            // the compositing loop (it would cost the kernel a resident wave
            // per SIMD).
            uint32_t ln;
            asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
#pragma unroll
            for (int q = 0; q < kPixPerLane; q++) {
                const int ryl = row0 + (int)(ln >> 4) + 4 * q;
                if (fy[q] != kInactiveRow)   // still compositing (so inside the region)
                    a.ckpt[(size_t)((rg.x + (uint32_t)b0) / kChunk) * (kTile * kTile) +
                           (uint32_t)(ryl * kTile) + (ln & 15)] = make_float4(T[q], cr[q], cg[q], cb[q]);
            }
            cuts_done++;
        }
        // Stage the entries that can reach 1/255 somewhere in this part's
        // rows, in list order; the others cannot change any of its pixels.
        const float u = rel_coord(g0.x, g0.z, px0), v = rel_coord(g0.y, g0.w, py0);
        const int k = b0 + lane;
        const uint32_t mask = k < len ? band_mask<kSplit>(u, v, g1.x, g1.y, g1.z, g1.w, row0) : 0u;
        const unsigned long long kept = __ballot(mask != 0u);
        const int nk = __popcll(kept);
        const bool nc_batch = __ballot(mask != 0u && !(g1.w <= kLoNoClamp)) == 0ull;
        if (mask != 0u) {
            const int r = kept_rank(kept);
            sA[r] = StagedA{u, v, g1.x, g1.y};
            sB[r] = StagedB{g1.z, g1.w, gc.x, gc.y};
            sF[r] = StagedF{gc.z, (uint32_t)k + 1u};
        }
        // padding up to the unroll width: inert records
        if (lane >= nk && lane < ((nk + kUnroll - 1) & ~(kUnroll - 1))) {
            sA[lane] = StagedA{0.f, 0.f, -1.f, 0.f};
            sB[lane] = StagedB{-1.f, -INFINITY, 0.f, 0.f};
            sF[lane] = StagedF{0.f, 0u};
        }
        __syncthreads();
        gather(b0 + kBatch + lane);
        // NC: no staged entry of the batch can reach the 0.99 clamp (same
        // alphas, one operation fewer per pixel); false once every pixel of
        // the part has stopped
        auto walk = [&](auto nc_c) __attribute__((always_inline)) {
            constexpr bool NC = decltype(nc_c)::value;
            for (int j0 = 0; j0 < nk; j0 += kUnroll) {
                StagedA es[kUnroll];
                StagedB et[kUnroll];
                StagedF ef[kUnroll];
    #pragma unroll
                for (int u2 = 0; u2 < kUnroll; u2++) {
                    es[u2] = sA[j0 + u2];
                    et[u2] = sB[j0 + u2];
                    ef[u2] = sF[j0 + u2];
                }
    #pragma unroll
                for (int u2 = 0; u2 < kUnroll; u2++) {
                    const int jp1 = (int)ef[u2].jp1;   // list position + 1
                    const ColTerms ct = col_terms(es[u2], fxl);
                    // hits: pixels still compositing (finite fy; the others get
                    // p2 = -inf and alpha = 0) with power <= 0 and alpha >= 1/255.
                    // (No separate p2 bound first: the staging cull already
                    // dropped the entries that reach 1/255 nowhere in these rows,
                    // and the backward's looser bound on p2 accepts every hit.)
                    float alpha[kPixPerLane];
                    bool hit[kPixPerLane];
                    bool any = false;
    #pragma unroll
                    for (int q = 0; q < kPixPerLane; q++) {
                        const float p2 = splat_p2(ct, et[u2].C2, es[u2].v - fy[q]);
                        const float apre = splat_alpha_pre(p2, et[u2].lo);
                        alpha[q] = NC ? apre : fminf(kAlphaMax, apre);   // NC: below the clamp
                        hit[q] = (p2 <= 0.f) & (alpha[q] >= kAlphaMin);
                        any |= hit[q];
                    }
                    // no pixel of this part reaches 1/255: nothing to do
                    if (!wave_any(any)) continue;
    #pragma unroll
                    for (int q = 0; q < kPixPerLane; q++) {
                        const float aT = alpha[q] * T[q];
                        const float testT = T[q] - aT;   // T (1 - alpha)
                        const bool blend = hit[q] && testT >= kTMin;
                        const bool stop = hit[q] && !(testT >= kTMin);
                        if (STATS) {
                            nb[q] += blend ? 1u : 0u;
                            ne[q] = stop ? (uint32_t)jp1 : ne[q];
                        }
                        const float wgt = blend ? aT : 0.f;
                        cr[q] = fmaf(et[u2].r, wgt, cr[q]);
                        cg[q] = fmaf(et[u2].g, wgt, cg[q]);
                        cb[q] = fmaf(ef[u2].b, wgt, cb[q]);
                        last[q] = blend ? jp1 : last[q];
                        T[q] = blend ? testT : T[q];
                        fy[q] = stop ? kInactiveRow : fy[q];
                    }
                }
                if (!any_active(fy)) return false;
            }
            return true;
        };
        const bool more = nc_batch ? walk(std::true_type{}) : walk(std::false_type{});
        if (!more) break;
        __syncthreads();
    }

    const int P = vw.roi_w * vw.roi_h;
    // L1-fused: sign(image - target) / (3 P), as gsp_loss_l1 writes it
    const float l1_inv = 1.0f / (float)(3 * (int64_t)P);
    double l1sum = 0.0;
#pragma unroll
    for (int q = 0; q < kPixPerLane; q++) {
        const int ry = kTile * ty + row0 + ly + 4 * q;
        if (rx >= vw.roi_w || ry >= vw.roi_h) continue;
        const size_t pix = (size_t)ry * vw.roi_w + rx;
        const float Tf = T[q];
        float *img = vw.img;
        const float fr = cr[q] + Tf * vw.bg[0], fg = cg[q] + Tf * vw.bg[1],
                    fb = cb[q] + Tf * vw.bg[2];
        if (a.l1) {
            const float *tg = vw.dl;
            const float c3[3] = {fr, fg, fb};
#pragma unroll
            for (int ch = 0; ch < 3; ch++) {
                const float d = c3[ch] - tg[(size_t)ch * P + pix];
                img[(size_t)ch * P + pix] = d > 0.f ? l1_inv : (d < 0.f ? -l1_inv : 0.f);
                l1sum += fabs((double)d);
            }
        } else {
            img[pix] = fr;
            img[(size_t)P + pix] = fg;
            img[2 * (size_t)P + pix] = fb;
        }
        if (last[q] > kChunk) {   // the backward's chunks derive the colour behind a cut from it
            a.cfinal[vw.pix_base + pix] = fr;
            a.cfinal[(size_t)a.total_pix + vw.pix_base + pix] = fg;
            a.cfinal[2 * (size_t)a.total_pix + vw.pix_base + pix] = fb;
        }
        a.tfinal[vw.pix_base + pix] = Tf;
        a.ncontrib[vw.pix_base + pix] = (uint32_t)last[q];
        if (vw.alpha) vw.alpha[pix] = 1.f - Tf;
        if (STATS) {
            // a pixel that never stopped evaluated the whole list
            a.neval[vw.pix_base + pix] = fy[q] == kInactiveRow ? ne[q] : (uint32_t)len;
            a.nblend[vw.pix_base + pix] = nb[q];
        }
    }
    if (a.l1part) {
        l1sum = wave_sum(l1sum);
        if (lane == 0) a.l1part[(size_t)tile * kSplit + part] = l1sum;
    }
}

// Loss of an L1-fused forward: per view, the waves' partial sums in tile and
// strip order, over the view's 3 x roi_h x roi_w values.
__global__ __launch_bounds__(256) void k_l1_fused_final(ViewsK views, const double *l1part,
                                                        float *loss) {
    __shared__ double red[256 / kWave];
    const ViewK &vw = views.v[blockIdx.x];
    const int64_t b0 = (int64_t)vw.tile_base * kSplit, n = (int64_t)vw.gw * vw.gh * kSplit;
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += 256) s += l1part[b0 + k];
    s = block_sum<double, 256>(s, red);
    if (threadIdx.x == 0) loss[blockIdx.x] = (float)(s / (double)(3 * (int64_t)vw.roi_w * vw.roi_h));
}

hipError_t launch_ranges(const Layout &L, char *ws, const uint32_t *keys, hipStream_t s) {
    uint2 *ranges = region<uint2>(ws, L.ranges);   // cleared by the emission
    const int64_t blocks = (L.cap + 255) / 256;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)blocks), dim3(256), 0, s, keys,
                       region<uint32_t>(ws, L.counters), ranges);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || L.total_tiles == 0) return e;
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, s, ranges, L.total_tiles,
                       region<uint32_t>(ws, L.tile_order), region<uint32_t>(ws, L.items),
                       region<uint32_t>(ws, L.counters));
    return hipGetLastError();
}

hipError_t launch_raster_fwd(const ViewsK &views, const Layout &L, char *ws, const uint32_t *vals,
                             bool stats, hipStream_t s, bool l1, float *loss) {
    if (L.total_tiles == 0) return hipSuccess;
    FwdArgs a;
    a.l1 = l1;
    a.l1part = l1 && loss ? region<double>(ws, L.l1part) : nullptr;
    a.order = region<uint32_t>(ws, L.tile_order);
    a.ranges = region<uint2>(ws, L.ranges);
    a.vals = vals;
    a.geom = region<float4>(ws, L.geom);
    a.color = region<float4>(ws, L.color);
    a.tfinal = region<float>(ws, L.tfinal);
    a.ncontrib = region<uint32_t>(ws, L.ncontrib);
    a.neval = region<uint32_t>(ws, L.stats);
    a.nblend = a.neval + L.total_pix;
    a.ckpt = region<float4>(ws, L.ckpt);
    a.cfinal = region<float>(ws, L.cfinal);
    a.total_pix = (int)L.total_pix;
    a.total_tiles = L.total_tiles;
    const dim3 grid(raster_blocks<kSplit>(L.total_tiles));
    if (stats)
        hipLaunchKernelGGL(k_raster_fwd<true>, grid, dim3(kRasterThreads), 0, s, a, views);
    else
        hipLaunchKernelGGL(k_raster_fwd<false>, grid, dim3(kRasterThreads), 0, s, a, views);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.l1part) return e;
    hipLaunchKernelGGL(k_l1_fused_final, dim3(views.count), dim3(256), 0, s, views, a.l1part, loss);
    return hipGetLastError();
}

}  // namespace gsp
