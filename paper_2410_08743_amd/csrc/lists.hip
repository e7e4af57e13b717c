// lists.hip -- the stored per-pixel state of the forward (GSP_STORE_LISTS).
//
// The default backward recomputes each pixel's compositing back to front
// from T_final, recovering T_i = T_{i+1} / (1 - alpha_i).  The stored mode
// instead keeps, after the forward, the list of every pixel's blended
// entries: for each blended splat i (front to back) its list position, its
// alpha (negated when the 0.99 clamp is active, which zeroes the derivative
// to the opacity and the power) and the transmittance T_i in front of it
// (Eq. (4)).  The stored backward then reads alpha_i and T_i instead of
// recomputing them.  This is the alternative the recomputing design avoids:
// 12 bytes per blended (pixel, splat) pair on top of the workspace.
//
// Three kernels over the tile lists the forward sorted: a counting pass of
// the list walk, an exclusive scan of the counts over all pixels, and the
// writing pass (the same walk, the same code, so both passes take the same
// decisions).  Each 16 x 16 tile is one 256-thread workgroup walking its
// list with one pixel per thread; the entries are broadcast loads (every
// thread of the tile reads the same record).
#include "block_ops.h"
#include "raster_common.h"

namespace gsp {

struct ListWalkArgs {
    const uint2 *ranges;
    const uint32_t *vals;
    const float4 *geom;
    const uint32_t *ncontrib;
    uint32_t *count;          // [total_pix] (counting pass)
    const uint32_t *offsets;  // [total_pix + 1] (writing pass)
    uint32_t *hdr;            // list header: pair count, overflow
    PairRec *pairs;
    int total_tiles;
};

// Walks the list of the tile of this workgroup for the thread's pixel up to
// its contributor count with the forward's per-entry arithmetic; WRITE = false
// counts the blended entries, WRITE = true stores them.
template <bool WRITE>
__global__ __launch_bounds__(256) void k_list_walk(ListWalkArgs a, ViewsK views) {
    const int tile = blockIdx.x;
    if (WRITE && a.hdr[kListOverflow]) return;
    const ViewK &vw = views.v[view_of_tile(views, tile)];
    const int lt = tile - vw.tile_base;
    const int tx = lt % vw.gw, ty = lt / vw.gw;
    const int px0 = vw.roi_x + kTile * tx, py0 = vw.roi_y + kTile * ty;
    const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
    const int rx = kTile * tx + lx, ry = kTile * ty + ly;
    const bool in = rx < vw.roi_w && ry < vw.roi_h;
    const size_t pix = (size_t)vw.pix_base + (size_t)ry * vw.roi_w + rx;
    const int last = in ? (int)a.ncontrib[pix] : 0;
    const uint2 rg = a.ranges[tile];
    uint32_t out = 0, end = 0;
    if (WRITE && in) {
        out = a.offsets[pix];
        end = a.offsets[pix + 1];
    }
    const float fxl = (float)lx, fyl = (float)ly;
    float T = 1.f;
    uint32_t n = 0;
    for (int k = 0; k < last; k++) {
        const uint32_t id = a.vals[rg.x + k];
        const float4 g0 = a.geom[2 * (size_t)id], g1 = a.geom[2 * (size_t)id + 1];
        const StagedA s{rel_coord(g0.x, g0.z, px0), rel_coord(g0.y, g0.w, py0), g1.x, g1.y};
        const ColTerms ct = col_terms(s, fxl);
        const float p2 = splat_p2(ct, g1.z, s.v - fyl);
        const float lim = kLog2AlphaMinLoose - g1.w;
        if (!((p2 <= 0.f) & (p2 >= lim))) continue;
        const float apre = splat_alpha_pre(p2, g1.w);
        const float alpha = fminf(kAlphaMax, apre);
        const float aT = alpha * T;
        const float testT = T - aT;
        if (!(alpha >= kAlphaMin && testT >= kTMin)) continue;
        if (WRITE) {
            if (out < end) a.pairs[out] = PairRec{(uint32_t)k, apre <= kAlphaMax ? alpha : -alpha, T};
            out++;
        }
        n++;
        T = testT;
    }
    if (!WRITE && in) a.count[pix] = n;
}

constexpr int kListScanItems = 1024;   // pixels per scan block

__global__ __launch_bounds__(256) void k_list_blocksums(const uint32_t *count, int total_pix,
                                                        unsigned long long *bs) {
    __shared__ unsigned long long red[256 / kWave];
    const int k0 = blockIdx.x * kListScanItems + 4 * threadIdx.x;
    unsigned long long c = 0;
#pragma unroll
    for (int j = 0; j < 4; j++)
        if (k0 + j < total_pix) c += count[k0 + j];
    c = block_sum<unsigned long long, 256>(c, red);
    if (threadIdx.x == 0) bs[blockIdx.x] = c;
}

// Exclusive offsets of the pixels' pair runs; each block sums the block sums
// in front of it itself.  Block 0 writes the total and the overflow flag
// (total above the pair capacity: the writing pass is skipped).
__global__ __launch_bounds__(256) void k_list_offsets(const uint32_t *count, int total_pix,
                                                      const unsigned long long *bs, int nblk,
                                                      unsigned long long capacity, uint32_t *offsets,
                                                      uint32_t *hdr) {
    __shared__ unsigned long long scratch[256 / kWave];
    const int t = threadIdx.x;
    unsigned long long before = 0, all = 0;
    for (int j = t; j < nblk; j += 256) {
        const unsigned long long x = bs[j];
        all += x;
        before += j < (int)blockIdx.x ? x : 0ull;
    }
    before = block_sum<unsigned long long, 256>(before, scratch);
    all = block_sum<unsigned long long, 256>(all, scratch);
    const bool ovf = all > capacity;
    if (blockIdx.x == 0 && t == 0) {
        hdr[kListPairsLo] = (uint32_t)(all & 0xffffffffull);
        hdr[kListPairsHi] = (uint32_t)(all >> 32);
        hdr[kListOverflow] = ovf ? 1u : 0u;
        if (ovf) hdr[kListSticky] = 1u;
    }
    if (ovf) return;
    const int k0 = blockIdx.x * kListScanItems + 4 * t;
    uint32_t c[4];
    unsigned long long local = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        c[j] = k0 + j < total_pix ? count[k0 + j] : 0u;
        local += c[j];
    }
    unsigned long long total;
    unsigned long long excl =
        block_exclusive_scan<unsigned long long, 256>(local, scratch, &total) + before;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        if (k0 + j >= total_pix) break;
        offsets[k0 + j] = (uint32_t)excl;
        excl += c[j];
        if (k0 + j == total_pix - 1) offsets[total_pix] = (uint32_t)excl;
    }
}

ListLayout make_list_layout(const Layout &L, int64_t pair_capacity) {
    ListLayout Q;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    Q.cap = pair_capacity;
    Q.nblk = (int)((L.total_pix + kListScanItems - 1) / kListScanItems);
    Q.hdr = take(kListHdrCount * 4);
    Q.count = take((size_t)L.total_pix * 4 + 4);
    Q.offsets = take(((size_t)L.total_pix + 1) * 4);
    Q.blocksum = take((size_t)(Q.nblk > 0 ? Q.nblk : 1) * 8);
    Q.pairs = take((size_t)(pair_capacity > 0 ? pair_capacity : 1) * kPairBytes);
    Q.total = off;
    return Q;
}

hipError_t launch_store_lists(const ViewsK &views, const Layout &L, char *ws, const uint32_t *vals,
                              const ListLayout &Q, char *lists, hipStream_t s) {
    // every call has at least one tile and one pixel (the views are validated)
    ListWalkArgs a;
    a.ranges = region<uint2>(ws, L.ranges);
    a.vals = vals;
    a.geom = region<float4>(ws, L.geom);
    a.ncontrib = region<uint32_t>(ws, L.ncontrib);
    a.count = region<uint32_t>(lists, Q.count);
    a.offsets = region<uint32_t>(lists, Q.offsets);
    a.hdr = region<uint32_t>(lists, Q.hdr);
    a.pairs = region<PairRec>(lists, Q.pairs);
    a.total_tiles = L.total_tiles;
    hipLaunchKernelGGL(k_list_walk<false>, dim3(L.total_tiles), dim3(256), 0, s, a, views);
    hipLaunchKernelGGL(k_list_blocksums, dim3(Q.nblk), dim3(256), 0, s, a.count, (int)L.total_pix,
                       region<unsigned long long>(lists, Q.blocksum));
    hipLaunchKernelGGL(k_list_offsets, dim3(Q.nblk), dim3(256), 0, s, a.count, (int)L.total_pix,
                       region<unsigned long long>(lists, Q.blocksum), Q.nblk,
                       (unsigned long long)Q.cap, region<uint32_t>(lists, Q.offsets), a.hdr);
    hipLaunchKernelGGL(k_list_walk<true>, dim3(L.total_tiles), dim3(256), 0, s, a, views);
    return hipGetLastError();
}

}  // namespace gsp
