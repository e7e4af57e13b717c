// gsp_internal.h -- internal declarations of the MI355X rasterizer library.
//
// Kernel-side constants, the per-call view table passed to kernels by value,
// the carving of the caller's workspace, and the host launchers of every
// kernel.  Nothing here is part of the public ABI (include/gsp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/gsp.h"

namespace gsp {

// ---------------------------------------------------------------------------
// Rasterizer constants.  The paper defers these to the 3DGS rasterizer it
// extends (Sec. III-A); the values are the readings fixed for this library.
// ---------------------------------------------------------------------------
constexpr int kTile = 16;                // tile edge in pixels
constexpr double kNear = 0.2;            // cull when camera-frame z <= near
constexpr double kDilation = 0.3;        // px^2 added to the 2D covariance diagonal
constexpr double kJClamp = 1.3;          // |x/z| clamp, in units of tan(fov/2)
constexpr double kLambdaFloor = 0.1;     // floor under the eigenvalue discriminant
constexpr float kAlphaMax = 0.99f;       // opacity clamp of a splat at a pixel
constexpr float kAlphaMin = 1.0f / 255.0f;  // splats below this alpha are skipped
constexpr float kTMin = 1e-4f;           // stop before transmittance drops below
constexpr double kLog2e = 1.4426950408889634;

constexpr int kPreprocessBlock = 256;    // Gaussians per preprocess block
constexpr int kSortThreads = 256;
// Keys per block of the instance sort (and per emission block): 1024, or
// 2048 above kSortLargeCap instances of capacity, where a 7-bit digit pass
// (more than 4096 tiles) would otherwise leave runs of 8 keys per digit and
// block, and the scatter's writes would cover half 64-byte segments
// (measured at 1M Gaussians, 4 views: tile sort 0.296 -> 0.233 ms; at one
// 1008 x 756 view the larger blocks cost 2 us).
constexpr int kSortRoundsSmall = 4, kSortRoundsLarge = 8;
constexpr int64_t kSortLargeCap = (int64_t)6 << 20;
inline int sort_items_for(int64_t cap) {
    return kSortThreads * (cap > kSortLargeCap ? kSortRoundsLarge : kSortRoundsSmall);
}
constexpr int kSortBits = 8;             // radix digit width
constexpr int kSortBins = 1 << kSortBits;
constexpr int kPoseReduceBlock = 256;
// Rows of per-wavefront pose partials per preprocess-backward block.
constexpr int kPoseRowsPerBlock = kPoseReduceBlock / 64;
// Instance-offset scan over the depth-sorted splats: splats per thread and
// per block.
constexpr int kScanPerThread = 4;
constexpr int kScanItems = kPreprocessBlock * kScanPerThread;
// Work windows of the instance emission and of the slot reduction: the
// sequence of splats in depth order, each followed by its instances, is cut
// into pieces of kWindow items, and a block takes the splats whose entry
// falls in its piece.  Every block then sees at most kWindow splats and
// kWindow instances plus the tail of its last splat, however unevenly the
// instances are spread over the splats.
#ifndef GSP_WINDOW
#define GSP_WINDOW 512
#endif
constexpr int kWindow = GSP_WINDOW;
constexpr int kWindowThreads = 256;
// Workgroups per 16 x 16 tile in the forward and per work item in the
// backward rasterizer (each takes a strip of 16 / split rows); every
// instance has one 9-float gradient slot per backward part.  The backward
// takes whole tiles (one wave, four pixels per lane): its chunked work
// items already fill the chip, and one wave per entry reduces the nine sums
// once instead of once per strip and halves the slots (measured: split 2
// 0.544 ms, split 1 0.503 ms per single-view step).
#ifndef GSP_SPLIT_FWD
#define GSP_SPLIT_FWD 4
#endif
#ifndef GSP_SPLIT_BWD
#define GSP_SPLIT_BWD 1
#endif
constexpr int kSplitFwd = GSP_SPLIT_FWD;
constexpr int kSplitBwd = GSP_SPLIT_BWD;
// Backward work items: a tile's list longer than kChunk entries is cut at
// multiples of kChunk into at most kMaxChunks chunks (the last one takes the
// rest), each walked by its own workgroups, so that no work item is long
// enough to run alone at the end of the launch (a 1008 x 756 view has 3024
// tiles of some 500 entries on average, for 4096 backward workgroup slots;
// 128 measured best among 64 .. 384).  The length is fixed, so a view is cut
// the same way alone or batched with others.  The forward records, per
// pixel, the transmittance and the accumulated colour at every cut, from
// which the backward of the chunk in front of the cut starts.  The cut at
// position p of the sorted instances has record p / kChunk: cuts are kChunk
// apart inside a list and more than that across lists, so no two share a
// record, and p < cap keeps the records below ceil(cap / kChunk).
#ifndef GSP_CHUNK
#define GSP_CHUNK 128
#endif
constexpr int kChunk = GSP_CHUNK;        // a multiple of the rasterizers' 64-entry batch
#ifndef GSP_MAX_CHUNKS
#define GSP_MAX_CHUNKS 16
#endif
constexpr int kMaxChunks = GSP_MAX_CHUNKS;
__host__ __device__ inline int chunks_of(int len) {
    const int c = (len + kChunk - 1) / kChunk;
    return c < 1 ? 1 : (c > kMaxChunks ? kMaxChunks : c);
}

// Per-view constants, computed on the host once per call.
struct ViewK {
    int W, H;
    float fx, fy, cx, cy;
    int roi_x, roi_y, roi_w, roi_h;
    int gw, gh;          // tile grid of the region of interest
    int tile_base;       // first global tile id of this view
    int pix_base;        // first pixel of this view in packed per-pixel arrays
    float bg[3];
    float *img;          // forward: the view's image, 3 x roi_h x roi_w
    float *alpha;        // forward: 1 - T_final per pixel, or null
    const float *dl;     // backward: dL/dimage, laid out like img
};

struct ViewsK {
    ViewK v[GSP_MAX_VIEWS];
    int count;
    int total_tiles;
};

// Carving of the caller's workspace.  Every region is 256-byte aligned.
struct Layout {
    int64_t n, vn, cap, total_pix;
    int32_t V, S, total_tiles, nblk_pre, nblk_scan, nblk_sort, nblk_emit, sort_items, tile_bits,
        tile_passes, nwin_max;
    // value bits of the instance sort's packed items (tile id above them),
    // or 0 when tile and value bits exceed 32 together (key and value arrays)
    int32_t sort_vbits;
    size_t geom, color, rect, depth, tiles, offsets, vis, offv, wstart, pstart, blocksum, blockvis,
        counters;
    size_t keys0, keys1, vals0, vals1, hist, digit_tot, ranges, tile_order;
    size_t items, ckpt, cfinal;   // backward work items, states at the cuts, final colours
    int64_t max_items;
    size_t tfinal, ncontrib, stats, slots, slot_flags, grad2d, posepart, l1part;
    size_t total;
};

// Counters at the start of the counters region.
// kCntSticky keeps the OR of every overflow since the workspace was zeroed;
// kCntWin is the number of work windows of this call; kCntItems the number of
// backward work items.
enum Counter : int {
    kCntMLo = 0, kCntMHi = 1, kCntOverflow = 2, kCntMEff = 3, kCntSticky = 4, kCntWin = 5,
    kCntItems = 6, kCntCount = 16
};

Layout make_layout(int64_t n, int32_t sh_degree, int32_t V, const ViewsK &views, int64_t cap);

// ---------------------------------------------------------------------------
// Launchers (each .hip file defines its own kernels and launchers).
// ---------------------------------------------------------------------------
struct GaussiansK {
    const float *means, *scales, *quats, *opacities, *sh;
    int n, sh_degree;
};

// lists.hip: the stored per-pixel state (GSP_STORE_LISTS).  A separate
// caller buffer: header | per-pixel counts | per-pixel offsets (+1) | scan
// block sums | pair records.
struct PairRec {
    uint32_t pos;     // list position in the tile
    float alpha;      // alpha_i, negated when clamped at 0.99
    float T;          // transmittance in front of i
};
constexpr int kPairBytes = 12;
static_assert(sizeof(PairRec) == kPairBytes, "pair record layout");
enum ListCounter : int {
    kListPairsLo = 0, kListPairsHi = 1, kListOverflow = 2, kListSticky = 3, kListHdrCount = 16
};
struct ListLayout {
    int64_t cap;
    int nblk;
    size_t hdr, count, offsets, blocksum, pairs, total;
};

// preprocess.hip
hipError_t launch_preprocess(const GaussiansK &g, const ViewsK &views, const float *poses,
                             const Layout &L, char *ws, hipStream_t s);
hipError_t launch_offsets_and_duplicate(const ViewsK &views, const Layout &L, char *ws,
                                        hipStream_t s);
// sort.hip
hipError_t launch_tile_sort(const Layout &L, char *ws, hipStream_t s);
hipError_t launch_tile_depth_sort(const Layout &L, char *ws, hipStream_t s);
// raster_fwd.hip
hipError_t launch_ranges(const Layout &L, char *ws, const uint32_t *keys, hipStream_t s);
// l1: each view's img receives dL/dimage of the L1 loss against the target
// its dl points to; with `loss`, the loss of each view goes there as well.
hipError_t launch_raster_fwd(const ViewsK &views, const Layout &L, char *ws,
                             const uint32_t *vals, bool stats, hipStream_t s, bool l1 = false,
                             float *loss = nullptr);
// raster_bwd.hip; with `lists` the stored-list variant (one workgroup per
// tile, alpha and T read from the pair records)
// want_opacity = false leaves the opacity component of every slot zero.
hipError_t launch_raster_bwd(const ViewsK &views, const Layout &L, char *ws,
                             const uint32_t *vals, bool want_opacity, hipStream_t s);
hipError_t launch_raster_bwd_stored(const ViewsK &views, const Layout &L, char *ws,
                                    const uint32_t *vals, const ListLayout &Q, const char *lists,
                                    hipStream_t s);
// lists.hip
ListLayout make_list_layout(const Layout &L, int64_t pair_capacity);
hipError_t launch_store_lists(const ViewsK &views, const Layout &L, char *ws, const uint32_t *vals,
                              const ListLayout &Q, char *lists, hipStream_t s);
// preprocess_bwd.hip
// Optional Adam step that the backward's final pose reduction applies to
// each view once its gradient is summed (the arguments of gsp_pose_adam;
// guard: the counters of the backward's workspace).
struct PoseAdamK {
    float *poses, *m, *v;
    int32_t *steps;
    gsp_adam_params p;
    const uint32_t *guard;
};
hipError_t launch_preprocess_bwd(const GaussiansK &g, const ViewsK &views, const float *poses,
                                 const Layout &L, char *ws, const gsp_grads &grads,
                                 bool accumulate, hipStream_t s, const PoseAdamK *adam = nullptr);
// misc.hip
struct LossViewsK {
    const float *pred[GSP_MAX_VIEWS];
    const float *target[GSP_MAX_VIEWS];
    float *grad[GSP_MAX_VIEWS];
    int64_t count[GSP_MAX_VIEWS];
    int64_t blk_base[GSP_MAX_VIEWS + 1];   // first loss block of each view
    int V;
};
constexpr int kLossItems = 4096;   // elements per loss block
int64_t loss_blocks(int64_t count);
hipError_t launch_loss_l1(const LossViewsK &lv, float *loss, void *partial_buf, hipStream_t s);
// Fixed per-device scratch of gsp_loss_l1_noalloc (bytes), and its device
// address on `device` (looked up once per device; thread-safe).
constexpr size_t kNoAllocScratchBytes = GSP_NOALLOC_SCRATCH_BYTES;
hipError_t noalloc_scratch_init(int device, void **ptr);
hipError_t launch_twist_apply(int V, const float *tau, const float *poses, float *out,
                              hipStream_t s);
hipError_t launch_twist_chain(int V, const float *tau, const float *g, float *out, hipStream_t s);
hipError_t launch_pose_adam(int V, float *poses, const float *dpose, float *m, float *v,
                            int32_t *steps, const gsp_adam_params &p, const uint32_t *guard,
                            hipStream_t s);

// joint.hip: L_RGB (Eq. (16)) over the views of a call, and Adam over the raw
// Gaussian parameters with the L_An hinge (Eq. (17)).
struct RgbViewsK {
    const float *pred[GSP_MAX_VIEWS];
    const float *target[GSP_MAX_VIEWS];
    float *grad[GSP_MAX_VIEWS];
    float *gmap[GSP_MAX_VIEWS];          // scratch: 3 maps x 3 channels x h x w
    int w[GSP_MAX_VIEWS], h[GSP_MAX_VIEWS], tiles_x[GSP_MAX_VIEWS];
    int tile_base[GSP_MAX_VIEWS + 1];    // first SSIM tile (per channel) of each view
    int V, total_tiles;
    float beta;
    float win[11];                       // normalised Gaussian window, sigma 1.5
};
int ssim_tiles(int w, int h);
hipError_t launch_loss_rgb(const RgbViewsK &a, float *loss, double2 *partial, hipStream_t s);

struct GaussAdamK {
    float *means, *log_scales, *quats, *logits, *sh;      // raw parameters, updated in place
    const float *g_means, *g_scales, *g_quats, *g_opacities, *g_sh;  // activated gradients
    float *m, *v;                        // moments, groups one after another
    float *scales_out, *opacities_out;   // activated values after the step
    double *partial;                     // L_An partial sums per block, or null
    const uint32_t *guard;               // counters of the producing render, or null
    int64_t n;
    int S;
    int64_t items[5];                    // cumulative work items: means, scales, quats, opacities, sh
    int64_t moff[5];                     // first moment of each group
    double lr_means, lr_scales, lr_quats, lr_opacities, lr_sh_dc, lr_sh_rest;
    double b1, b2, c1, c2, eps;
    double aniso_r, aniso_w;
};
int64_t gauss_adam_partials(int64_t n);
hipError_t launch_gauss_adam(const GaussAdamK &a, float *aniso_loss, hipStream_t s);

// relpose.hip: scene of frame t from its depth map, and the masked L1
// (Sec. III-D, Eq. (20)-(21)).
constexpr int kMaxUnprojectPoints = 1 << 18;   // n^2 neighbour tests: ~2 s at the limit
struct UnprojK {
    const float *depth, *image;          // [h][w], [3][h][w] over the region of interest
    int w, h, stride, nx, ny, S, roi_x, roi_y;
    float fx, fy, cx, cy, logit;
    float *means, *log_scales, *quats, *logits, *sh;   // raw parameters out
    float4 *pts;                         // scratch: (x, y, z, valid) per point
};
hipError_t launch_unproject(const UnprojK &a, hipStream_t s);

struct MaskViewsK {
    const float *pred[GSP_MAX_VIEWS];
    const float *target[GSP_MAX_VIEWS];
    const float *alpha[GSP_MAX_VIEWS];
    float *grad[GSP_MAX_VIEWS];
    int64_t pix[GSP_MAX_VIEWS];
    int64_t blk_base[GSP_MAX_VIEWS + 1];
    int V;
};
int64_t masked_blocks(int64_t count);
hipError_t launch_masked_l1(const MaskViewsK &a, float *loss, void *scratch, hipStream_t s);

template <typename T>
inline T *region(char *ws, size_t off) { return reinterpret_cast<T *>(ws + off); }

inline int tile_bits_for(int total_tiles) {
    int tile_bits = 0;
    while ((1ll << tile_bits) < (long long)total_tiles) tile_bits++;
    return tile_bits;
}

// Passes of a radix sort on `bits` key bits, and the digit width of each:
// the bits are shared out evenly (12 bits: two 6-bit passes rather than 8 +
// 4), which keeps the digit runs of the first pass long enough for
// full-line stores.
inline int sort_passes(int bits) { return (bits + kSortBits - 1) / kSortBits; }
inline int digit_bits(int bits) {
    const int p = sort_passes(bits);
    return p > 0 ? (bits + p - 1) / p : 0;
}

// Buffers holding the result of the two sorts (depth: 4 passes, even).
inline size_t sorted_keys(const Layout &L) { return (L.tile_passes & 1) ? L.keys1 : L.keys0; }
inline size_t sorted_vals(const Layout &L) { return (L.tile_passes & 1) ? L.vals1 : L.vals0; }

}  // namespace gsp
