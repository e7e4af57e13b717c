// api.hip -- the C ABI of include/gsp.h: argument validation, the per-call
// view table, workspace carving and the launch sequence of the forward and
// backward passes.  Host code only; every step of the path runs in the
// kernels of the other files.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gsp_internal.h"

namespace {
struct StageRec {
    const char *name;
    hipEvent_t start, stop;
};
struct StageSum {
    std::string name;
    int64_t count;
    double ms;
};
}  // namespace

struct gsp_ctx {
    int device;
    void *noalloc_scratch = nullptr;   // device address of the library's fixed L1 scratch
    bool profiling = false;   // stage timing
    bool stats = false;       // per-pixel work counters in the forward
    std::vector<StageRec> pending;
    std::vector<hipEvent_t> pool;
    std::vector<StageSum> sums;
};

namespace {

thread_local std::string g_last_error;

gsp_status fail(gsp_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
gsp_status fail(gsp_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

gsp_status hip_fail(hipError_t e, const char *where) {
    return fail(GSP_EHIP, "%s: %s", where, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

hipEvent_t take_event(gsp_ctx *ctx) {
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs one stage's launcher, bracketed by events when profiling is on.
template <typename F>
hipError_t stage(gsp_ctx *ctx, const char *name, hipStream_t st, F &&launch) {
    if (!ctx->profiling) return launch();
    StageRec r{name, take_event(ctx), take_event(ctx)};
    if (r.start) hipEventRecord(r.start, st);
    hipError_t e = launch();
    if (r.stop) hipEventRecord(r.stop, st);
    if (r.start && r.stop) ctx->pending.push_back(r);
    return e;
}

gsp_status check_device(const gsp_ctx *ctx) {
    if (!ctx) return fail(GSP_EINVAL, "null context");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != ctx->device)
        return fail(GSP_EINVAL, "current device %d differs from the context's device %d", dev,
                    ctx->device);
    return GSP_OK;
}

// Validates the views and fills the kernel view table.
gsp_status make_views(int32_t V, const gsp_view *views, gsp::ViewsK *out, int64_t *total_pix) {
    if (V < 1 || V > GSP_MAX_VIEWS)
        return fail(GSP_EINVAL, "view count %d outside 1..%d", V, GSP_MAX_VIEWS);
    if (!views) return fail(GSP_EINVAL, "null views");
    std::memset(out, 0, sizeof *out);
    int64_t tiles = 0, pix = 0;
    for (int v = 0; v < V; v++) {
        const gsp_view &w = views[v];
        if (w.width <= 0 || w.height <= 0 || w.width > 65535 * gsp::kTile ||
            w.height > 65535 * gsp::kTile)
            return fail(GSP_EINVAL, "view %d: bad image size %dx%d", v, w.width, w.height);
        if (!(w.fx > 0.f) || !(w.fy > 0.f) || !std::isfinite(w.cx) || !std::isfinite(w.cy))
            return fail(GSP_EINVAL, "view %d: bad intrinsics", v);
        if (w.roi_x < 0 || w.roi_y < 0 || w.roi_w <= 0 || w.roi_h <= 0 ||
            w.roi_x % gsp::kTile || w.roi_y % gsp::kTile || w.roi_x + w.roi_w > w.width ||
            w.roi_y + w.roi_h > w.height)
            return fail(GSP_EINVAL,
                        "view %d: region of interest (%d,%d,%d,%d) must start on a multiple of "
                        "16 and lie inside the %dx%d image",
                        v, w.roi_x, w.roi_y, w.roi_w, w.roi_h, w.width, w.height);
        gsp::ViewK &k = out->v[v];
        k.W = w.width;
        k.H = w.height;
        k.fx = w.fx;
        k.fy = w.fy;
        k.cx = w.cx;
        k.cy = w.cy;
        k.roi_x = w.roi_x;
        k.roi_y = w.roi_y;
        k.roi_w = w.roi_w;
        k.roi_h = w.roi_h;
        k.gw = (w.roi_w + gsp::kTile - 1) / gsp::kTile;
        k.gh = (w.roi_h + gsp::kTile - 1) / gsp::kTile;
        k.tile_base = (int)tiles;
        k.pix_base = (int)pix;
        for (int c = 0; c < 3; c++) k.bg[c] = w.bg[c];
        tiles += (int64_t)k.gw * k.gh;
        pix += (int64_t)w.roi_w * w.roi_h;
    }
    if (tiles >= (1ll << 31) || pix >= (1ll << 31))
        return fail(GSP_EINVAL, "too many tiles or pixels in one call");
    out->count = V;
    out->total_tiles = (int)tiles;
    *total_pix = pix;
    return GSP_OK;
}

gsp_status check_gaussians(const gsp_gaussians *g, int32_t V) {
    if (!g) return fail(GSP_EINVAL, "null Gaussians");
    if (g->n < 0 || g->n * (int64_t)V >= (1ll << 31))
        return fail(GSP_EINVAL, "Gaussian count %lld too large for %d views", (long long)g->n, V);
    if (g->sh_degree < 0 || g->sh_degree > 3)
        return fail(GSP_EINVAL, "sh_degree %d outside 0..3", g->sh_degree);
    if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacities || !g->sh))
        return fail(GSP_EINVAL, "null Gaussian parameter array");
    return GSP_OK;
}

gsp::GaussiansK kernel_gaussians(const gsp_gaussians *g) {
    gsp::GaussiansK k;
    k.means = g->means;
    k.scales = g->scales;
    k.quats = g->quats;
    k.opacities = g->opacities;
    k.sh = g->sh;
    k.n = (int)g->n;
    k.sh_degree = g->sh_degree;
    return k;
}

struct Prepared {
    gsp::ViewsK views;
    gsp::Layout L;
};

gsp_status prepare(const gsp_gaussians *g, int32_t V, const gsp_view *views, int64_t cap,
                   Prepared *p) {
    gsp_status s = check_gaussians(g, V);
    if (s != GSP_OK) return s;
    int64_t total_pix = 0;
    s = make_views(V, views, &p->views, &total_pix);
    if (s != GSP_OK) return s;
    if (cap < 0 || cap >= (1ll << 32) - 1)
        return fail(GSP_EINVAL, "instance capacity %lld outside 0..2^32-2", (long long)cap);
    p->L = gsp::make_layout(g->n, g->sh_degree, V, p->views, cap);
    return GSP_OK;
}

}  // namespace

namespace gsp {

Layout make_layout(int64_t n, int32_t sh_degree, int32_t V, const ViewsK &views, int64_t cap) {
    Layout L;
    std::memset(&L, 0, sizeof L);
    L.n = n;
    L.V = V;
    L.vn = n * V;
    L.S = (sh_degree + 1) * (sh_degree + 1);
    L.cap = cap > 0 ? cap : 1;
    L.total_tiles = views.total_tiles;
    int64_t pix = 0;
    for (int v = 0; v < V; v++) pix += (int64_t)views.v[v].roi_w * views.v[v].roi_h;
    L.total_pix = pix;
    L.nblk_pre = (int)((n + kPreprocessBlock - 1) / kPreprocessBlock);
    L.nblk_scan = (int)((L.vn + kScanItems - 1) / kScanItems);
    L.sort_items = sort_items_for(L.cap);
    L.nblk_sort = (int)((L.cap + L.sort_items - 1) / L.sort_items);
    L.nblk_emit = L.nblk_sort;   // emission blocks are the instance sort's first-pass blocks
    L.tile_bits = tile_bits_for(views.total_tiles);
    {
        // packed instance-sort items when the tile id and the value fit one word
        const int vbits = L.vn > 1 ? 64 - __builtin_clzll((unsigned long long)(L.vn - 1)) : 1;
        L.sort_vbits = L.tile_bits > 0 && L.tile_bits + vbits <= 32 ? vbits : 0;
    }
    L.tile_passes = sort_passes(L.tile_bits);
    L.nwin_max = (int)((L.vn + L.cap + kWindow - 1) / kWindow + 1);
    const size_t vn = (size_t)L.vn, capz = (size_t)L.cap;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes > 0 ? bytes : 1);
        return o;
    };
    L.counters = take(kCntCount * 4);   // first, so that gsp_instances needs no sizes
    L.geom = take(vn * 32);
    L.color = take(vn * 16);
    L.rect = take(vn * 8);
    L.depth = take(vn * 4);
    L.tiles = take(vn * 4);
    L.offsets = take((vn + 1) * 4);
    L.vis = take(vn * 4);
    L.offv = take((vn + 1) * 4);
    L.wstart = take(((size_t)L.nwin_max + 1) * 8);
    L.pstart = take(((size_t)L.nblk_emit + 1) * 4);
    L.blocksum = take((size_t)L.nblk_scan * 8 + 8);
    L.blockvis = take((size_t)L.nblk_scan * 4 + 4);
    L.keys0 = take(capz * 4);
    L.keys1 = take(capz * 4);
    L.vals0 = take(capz * 4);
    L.vals1 = take(capz * 4);
    L.hist = take((size_t)kSortBins * L.nblk_sort * 4);
    L.digit_tot = take((size_t)kSortBins * 4);
    L.ranges = take((size_t)L.total_tiles * 8);
    L.tile_order = take((size_t)L.total_tiles * 4);
    // Every chunk in front of a cut holds kChunk entries, so there are at
    // most cap / kChunk cuts and one work item per tile more than that; a
    // cut at sorted position p < cap has record p / kChunk.
    L.max_items = (int64_t)L.total_tiles + (int64_t)(capz / kChunk);
    L.items = take((size_t)L.max_items * 4);
    L.ckpt = take((capz + kChunk - 1) / kChunk * kTile * kTile * 16);
    L.cfinal = take((size_t)pix * 12);
    L.tfinal = take((size_t)pix * 4);
    L.ncontrib = take((size_t)pix * 4);
    L.stats = take((size_t)pix * 8);
    L.slots = take(9 * (size_t)kSplitBwd * capz * 4);
    L.slot_flags = take(((size_t)kSplitBwd * capz + 3) & ~size_t(3));
    L.grad2d = take(9 * vn * 4);
    L.posepart = take((size_t)V * L.nblk_pre * kPoseRowsPerBlock * 6 * 8);
    L.l1part = take((size_t)L.total_tiles * kSplitFwd * 8);
    L.total = off;
    return L;
}

}  // namespace gsp

extern "C" {

int gsp_version(void) { return 1; }

const char *gsp_status_string(gsp_status s) {
    switch (s) {
        case GSP_OK: return "ok";
        case GSP_EINVAL: return "invalid argument";
        case GSP_ECAPACITY: return "instance capacity exceeded";
        case GSP_ENOMEM: return "workspace too small";
        case GSP_EHIP: return "HIP runtime error";
        case GSP_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *gsp_last_error(void) { return g_last_error.c_str(); }

gsp_status gsp_create(int device, gsp_ctx **out) {
    if (!out) return fail(GSP_EINVAL, "null output pointer");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count)
        return fail(GSP_EINVAL, "device %d outside 0..%d", device, count - 1);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(GSP_EUNSUPPORTED, "device %d is %s; this library is built for gfx950", device,
                    prop.gcnArchName);
    void *scratch = nullptr;
    e = gsp::noalloc_scratch_init(device, &scratch);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the fixed scratch");
    gsp_ctx *ctx = new (std::nothrow) gsp_ctx;
    if (!ctx) return fail(GSP_ENOMEM, "out of host memory");
    ctx->device = device;
    ctx->noalloc_scratch = scratch;
    *out = ctx;
    return GSP_OK;
}

gsp_status gsp_destroy(gsp_ctx *ctx) {
    if (!ctx) return GSP_OK;
    for (StageRec &r : ctx->pending) {
        hipEventSynchronize(r.stop);
        hipEventDestroy(r.start);
        hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : ctx->pool) hipEventDestroy(e);
    delete ctx;
    return GSP_OK;
}

gsp_status gsp_profile_enable(gsp_ctx *ctx, int mode) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    if (mode & ~(GSP_PROFILE_TIMING | GSP_PROFILE_COUNTS)) return fail(GSP_EINVAL, "bad mode");
    ctx->profiling = (mode & GSP_PROFILE_TIMING) != 0;
    ctx->stats = (mode & GSP_PROFILE_COUNTS) != 0;
    return GSP_OK;
}

gsp_status gsp_profile_read(gsp_ctx *ctx, int32_t max_stages, char *names, int64_t *counts,
                            double *ms, int32_t *n_out) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    if (max_stages < 0 || (max_stages > 0 && (!names || !counts || !ms)) || !n_out)
        return fail(GSP_EINVAL, "bad profile output arguments");
    for (StageRec &r : ctx->pending) {
        hipError_t e = hipEventSynchronize(r.stop);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float t = 0.f;
        e = hipEventElapsedTime(&t, r.start, r.stop);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        StageSum *sum = nullptr;
        for (StageSum &x : ctx->sums)
            if (x.name == r.name) sum = &x;
        if (!sum) {
            ctx->sums.push_back(StageSum{r.name, 0, 0.0});
            sum = &ctx->sums.back();
        }
        sum->count += 1;
        sum->ms += t;
        ctx->pool.push_back(r.start);
        ctx->pool.push_back(r.stop);
    }
    ctx->pending.clear();
    int32_t k = 0;
    for (const StageSum &x : ctx->sums) {
        if (k >= max_stages) break;
        std::snprintf(names + 32 * k, 32, "%s", x.name.c_str());
        counts[k] = x.count;
        ms[k] = x.ms;
        k++;
    }
    *n_out = k;
    ctx->sums.clear();
    return GSP_OK;
}

gsp_status gsp_workspace_size(int64_t n, int32_t sh_degree, int32_t V, const gsp_view *views,
                              int64_t instance_capacity, size_t *bytes) {
    if (!bytes) return fail(GSP_EINVAL, "null output pointer");
    gsp_gaussians g;
    std::memset(&g, 0, sizeof g);
    g.n = n;
    g.sh_degree = sh_degree;
    if (n < 0 || sh_degree < 0 || sh_degree > 3) return fail(GSP_EINVAL, "bad n or sh_degree");
    Prepared p;
    int64_t total_pix;
    gsp_status s = make_views(V, views, &p.views, &total_pix);
    if (s != GSP_OK) return s;
    if (instance_capacity < 0 || instance_capacity >= (1ll << 32) - 1)
        return fail(GSP_EINVAL, "instance capacity out of range");
    *bytes = gsp::make_layout(n, sh_degree, V, p.views, instance_capacity).total;
    return GSP_OK;
}

namespace {

gsp_status check_lists(const gsp::Layout &L, const void *lists, size_t lists_bytes,
                       int64_t pair_capacity, gsp::ListLayout *Q) {
    if (!lists) return fail(GSP_EINVAL, "null list buffer");
    if (pair_capacity < 0 || pair_capacity >= (1ll << 32) - 1)
        return fail(GSP_EINVAL, "pair capacity %lld outside 0..2^32-2", (long long)pair_capacity);
    *Q = gsp::make_list_layout(L, pair_capacity);
    if (lists_bytes < Q->total)
        return fail(GSP_ENOMEM, "list buffer of %zu bytes is smaller than the %zu needed",
                    lists_bytes, Q->total);
    return GSP_OK;
}

// With targets, the forward writes dL/dimage of the per-view L1 loss into
// `images` (the gradient buffers) instead of the images, and the losses into
// `loss` when it is given.
gsp_status render_fwd(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V, const gsp_view *views,
                      const float *poses, float *const *images, float *const *alphas,
                      void *workspace, size_t ws_bytes, int64_t instance_capacity, void *lists,
                      size_t lists_bytes, int64_t pair_capacity, void *stream,
                      const float *const *targets = nullptr, float *loss = nullptr) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    Prepared p;
    s = prepare(g, V, views, instance_capacity, &p);
    if (s != GSP_OK) return s;
    if (!poses || !images || !workspace) return fail(GSP_EINVAL, "null poses, images or workspace");
    for (int v = 0; v < V; v++) {
        if (!images[v]) return fail(GSP_EINVAL, "null image pointer of view %d", v);
        p.views.v[v].img = images[v];
        p.views.v[v].alpha = alphas ? alphas[v] : nullptr;
        if (targets) {
            if (!targets[v]) return fail(GSP_EINVAL, "null target pointer of view %d", v);
            p.views.v[v].dl = targets[v];   // the forward reads the target through dl
        }
    }
    if (ws_bytes < p.L.total)
        return fail(GSP_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes,
                    p.L.total);
    gsp::ListLayout Q;
    std::memset(&Q, 0, sizeof Q);
    if (lists && (s = check_lists(p.L, lists, lists_bytes, pair_capacity, &Q)) != GSP_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    const gsp::GaussiansK gk = kernel_gaussians(g);
    hipError_t e;
    if ((e = stage(ctx, "preprocess", st, [&] {
             return gsp::launch_preprocess(gk, p.views, poses, p.L, ws, st);
         })) != hipSuccess)
        return hip_fail(e, "preprocess");
    if ((e = stage(ctx, "duplicate", st, [&] {
             return gsp::launch_offsets_and_duplicate(p.views, p.L, ws, st);
         })) != hipSuccess)
        return hip_fail(e, "duplicate");
    if ((e = stage(ctx, "tile_sort", st, [&] { return gsp::launch_tile_sort(p.L, ws, st); })) !=
        hipSuccess)
        return hip_fail(e, "tile sort");
    const uint32_t *keys = gsp::region<uint32_t>(ws, gsp::sorted_keys(p.L));
    const uint32_t *vals = gsp::region<uint32_t>(ws, gsp::sorted_vals(p.L));
    if ((e = stage(ctx, "ranges", st, [&] { return gsp::launch_ranges(p.L, ws, keys, st); })) !=
        hipSuccess)
        return hip_fail(e, "ranges");
    if ((e = stage(ctx, "depth_order", st, [&] { return gsp::launch_tile_depth_sort(p.L, ws, st); })) !=
        hipSuccess)
        return hip_fail(e, "depth order");
    if ((e = stage(ctx, "raster_fwd", st, [&] {
             return gsp::launch_raster_fwd(p.views, p.L, ws, vals, ctx->stats, st, targets != nullptr,
                                           loss);
         })) != hipSuccess)
        return hip_fail(e, "raster forward");
    if (lists) {
        if ((e = stage(ctx, "store_lists", st, [&] {
                 return gsp::launch_store_lists(p.views, p.L, ws, vals, Q, static_cast<char *>(lists),
                                                st);
             })) != hipSuccess)
            return hip_fail(e, "store lists");
    }
    return GSP_OK;
}

}  // namespace

gsp_status gsp_render_fwd(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V, const gsp_view *views,
                          const float *poses, float *const *images, float *const *alphas,
                          void *workspace, size_t ws_bytes, int64_t instance_capacity,
                          void *stream) {
    return render_fwd(ctx, g, V, views, poses, images, alphas, workspace, ws_bytes,
                      instance_capacity, nullptr, 0, 0, stream);
}

gsp_status gsp_render_fwd_l1(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V,
                             const gsp_view *views, const float *poses,
                             const float *const *targets, float *const *dl_dimages,
                             float *const *alphas, float *loss, void *workspace, size_t ws_bytes,
                             int64_t instance_capacity, void *stream) {
    if (!targets || !dl_dimages) return fail(GSP_EINVAL, "null targets or gradients");
    return render_fwd(ctx, g, V, views, poses, dl_dimages, alphas, workspace, ws_bytes,
                      instance_capacity, nullptr, 0, 0, stream, targets, loss);
}

gsp_status gsp_render_fwd_store(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V,
                                const gsp_view *views, const float *poses, float *const *images,
                                float *const *alphas, void *workspace, size_t ws_bytes,
                                int64_t instance_capacity, void *lists, size_t lists_bytes,
                                int64_t pair_capacity, void *stream) {
    if (!lists) return fail(GSP_EINVAL, "null list buffer");
    return render_fwd(ctx, g, V, views, poses, images, alphas, workspace, ws_bytes,
                      instance_capacity, lists, lists_bytes, pair_capacity, stream);
}

size_t gsp_lists_bytes(int32_t V, const gsp_view *views, int64_t pair_capacity) {
    gsp::ViewsK vk;
    int64_t total_pix = 0;
    if (make_views(V, views, &vk, &total_pix) != GSP_OK) return 0;
    if (pair_capacity < 0 || pair_capacity >= (1ll << 32) - 1) return 0;
    const gsp::Layout L = gsp::make_layout(0, 0, V, vk, 0);
    return gsp::make_list_layout(L, pair_capacity).total;
}

gsp_status gsp_list_pairs(gsp_ctx *ctx, const void *lists, void *stream, int64_t *pairs_out,
                          int32_t *overflow_out) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    if (!lists) return fail(GSP_EINVAL, "null list buffer");
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    uint32_t c[gsp::kListHdrCount];
    e = hipMemcpy(c, lists, sizeof c, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    if (pairs_out) *pairs_out = (int64_t)(((uint64_t)c[gsp::kListPairsHi] << 32) | c[gsp::kListPairsLo]);
    if (overflow_out) *overflow_out = (int32_t)(c[gsp::kListOverflow] | c[gsp::kListSticky]);
    return GSP_OK;
}

namespace {

gsp_status render_bwd(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V, const gsp_view *views,
                      const float *poses, const float *const *dl_dimages, void *workspace,
                      size_t ws_bytes, int64_t instance_capacity, const void *lists,
                      size_t lists_bytes, int64_t pair_capacity, const gsp_grads *grads,
                      uint32_t flags, void *stream, const gsp::PoseAdamK *adam = nullptr) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    Prepared p;
    s = prepare(g, V, views, instance_capacity, &p);
    if (s != GSP_OK) return s;
    if (!poses || !dl_dimages || !workspace || !grads)
        return fail(GSP_EINVAL, "null poses, dl_dimages, workspace or grads");
    for (int v = 0; v < V; v++) {
        if (!dl_dimages[v]) return fail(GSP_EINVAL, "null dl_dimages pointer of view %d", v);
        p.views.v[v].dl = dl_dimages[v];
    }
    if (flags & ~GSP_ACCUMULATE) return fail(GSP_EINVAL, "unknown flags 0x%x", flags);
    if (ws_bytes < p.L.total)
        return fail(GSP_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes,
                    p.L.total);
    gsp::ListLayout Q;
    std::memset(&Q, 0, sizeof Q);
    if (lists && (s = check_lists(p.L, lists, lists_bytes, pair_capacity, &Q)) != GSP_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    const uint32_t *vals = gsp::region<uint32_t>(ws, gsp::sorted_vals(p.L));
    hipError_t e;
    if ((e = stage(ctx, "raster_bwd", st, [&] {
             return lists ? gsp::launch_raster_bwd_stored(p.views, p.L, ws, vals, Q,
                                                          static_cast<const char *>(lists), st)
                          : gsp::launch_raster_bwd(p.views, p.L, ws, vals, grads->opacities != nullptr,
                                                   st);
         })) != hipSuccess)
        return hip_fail(e, "raster backward");
    if ((e = stage(ctx, "preprocess_bwd", st, [&] {
             return gsp::launch_preprocess_bwd(kernel_gaussians(g), p.views, poses, p.L, ws, *grads,
                                               (flags & GSP_ACCUMULATE) != 0, st, adam);
         })) != hipSuccess)
        return hip_fail(e, "preprocess backward");
    return GSP_OK;
}

}  // namespace

gsp_status gsp_render_bwd(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V, const gsp_view *views,
                          const float *poses, const float *const *dl_dimages, void *workspace,
                          size_t ws_bytes, int64_t instance_capacity, const gsp_grads *grads,
                          uint32_t flags, void *stream) {
    return render_bwd(ctx, g, V, views, poses, dl_dimages, workspace, ws_bytes, instance_capacity,
                      nullptr, 0, 0, grads, flags, stream);
}

gsp_status gsp_render_bwd_pose_step(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V,
                                    const gsp_view *views, float *poses,
                                    const float *const *dl_dimages, void *workspace, size_t ws_bytes,
                                    int64_t instance_capacity, float *dpose, float *m, float *v,
                                    int32_t *steps, const gsp_adam_params *params, void *stream) {
    if (!poses || !dpose || !m || !v || !steps || !params) return fail(GSP_EINVAL, "null argument");
    if (!(params->beta1 >= 0.f && params->beta1 < 1.f && params->beta2 >= 0.f &&
          params->beta2 < 1.f && params->eps > 0.f))
        return fail(GSP_EINVAL, "bad Adam hyper-parameters");
    if (params->parametrization != GSP_POSE_SE3 && params->parametrization != GSP_POSE_T_SO3)
        return fail(GSP_EINVAL, "unknown pose parametrization %d", params->parametrization);
    if (!workspace) return fail(GSP_EINVAL, "null workspace");
    gsp_grads grads;
    std::memset(&grads, 0, sizeof grads);
    grads.pose = dpose;
    gsp::PoseAdamK ad;
    ad.poses = poses;
    ad.m = m;
    ad.v = v;
    ad.steps = steps;
    ad.p = *params;
    ad.guard = static_cast<const uint32_t *>(workspace);   // the counters open the workspace
    return render_bwd(ctx, g, V, views, poses, dl_dimages, workspace, ws_bytes, instance_capacity,
                      nullptr, 0, 0, &grads, 0u, stream, &ad);
}

gsp_status gsp_render_bwd_stored(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V,
                                 const gsp_view *views, const float *poses,
                                 const float *const *dl_dimages, void *workspace, size_t ws_bytes,
                                 int64_t instance_capacity, const void *lists, size_t lists_bytes,
                                 int64_t pair_capacity, const gsp_grads *grads, uint32_t flags,
                                 void *stream) {
    if (!lists) return fail(GSP_EINVAL, "null list buffer");
    return render_bwd(ctx, g, V, views, poses, dl_dimages, workspace, ws_bytes, instance_capacity,
                      lists, lists_bytes, pair_capacity, grads, flags, stream);
}

gsp_status gsp_instances(gsp_ctx *ctx, const void *workspace, void *stream, int64_t *m_out,
                         int32_t *overflow_out) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    if (!workspace) return fail(GSP_EINVAL, "null workspace");
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    uint32_t c[gsp::kCntCount];
    e = hipMemcpy(c, workspace, sizeof c, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    if (m_out) *m_out = (int64_t)(((uint64_t)c[gsp::kCntMHi] << 32) | c[gsp::kCntMLo]);
    if (overflow_out) *overflow_out = (int32_t)(c[gsp::kCntOverflow] | c[gsp::kCntSticky]);
    return GSP_OK;
}

gsp_status gsp_inspect(gsp_ctx *ctx, const gsp_gaussians *g, int32_t V, const gsp_view *views,
                       void *workspace, size_t ws_bytes, int64_t instance_capacity,
                       const char *name, void **ptr, int64_t *count) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    Prepared p;
    s = prepare(g, V, views, instance_capacity, &p);
    if (s != GSP_OK) return s;
    if (!workspace || !name || !ptr || !count) return fail(GSP_EINVAL, "null argument");
    if (ws_bytes < p.L.total) return fail(GSP_ENOMEM, "workspace too small for these sizes");
    const gsp::Layout &L = p.L;
    char *ws = static_cast<char *>(workspace);
    struct Entry { const char *n; size_t off; int64_t cnt; };
    const Entry table[] = {
        {"geom", L.geom, 2 * L.vn},
        {"color", L.color, L.vn},
        {"rect", L.rect, L.vn},
        {"depth", L.depth, L.vn},
        {"tiles", L.tiles, L.vn},
        {"offsets", L.offsets, L.vn},
        {"keys", gsp::sorted_keys(L), L.cap},
        {"values", gsp::sorted_vals(L), L.cap},
        {"ranges", L.ranges, L.total_tiles},
        {"tfinal", L.tfinal, L.total_pix},
        {"ncontrib", L.ncontrib, L.total_pix},
        {"neval", L.stats, L.total_pix},
        {"nblend", L.stats + 4 * (size_t)L.total_pix, L.total_pix},
        {"grad2d", L.grad2d, 9 * L.vn},
        {"counters", L.counters, gsp::kCntCount},
    };
    for (const Entry &en : table) {
        if (std::strcmp(en.n, name) == 0) {
            *ptr = ws + en.off;
            *count = en.cnt;
            return GSP_OK;
        }
    }
    return fail(GSP_EINVAL, "unknown workspace array \"%s\"", name);
}

gsp_status gsp_loss_l1(gsp_ctx *ctx, int32_t V, const gsp_view *views, const float *const *pred,
                       const float *const *target, float *const *grad, float *loss,
                       void *scratch, void *stream) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    gsp::ViewsK vk;
    int64_t total_pix = 0;
    s = make_views(V, views, &vk, &total_pix);
    if (s != GSP_OK) return s;
    if (!pred || !target || !grad) return fail(GSP_EINVAL, "null pointer array");
    if (loss && !scratch) return fail(GSP_EINVAL, "loss requires scratch memory");
    gsp::LossViewsK lv;
    std::memset(&lv, 0, sizeof lv);
    lv.V = V;
    lv.blk_base[0] = 0;
    for (int v = 0; v < V; v++) {
        if (!pred[v] || !target[v] || !grad[v])
            return fail(GSP_EINVAL, "null pred, target or grad of view %d", v);
        lv.pred[v] = pred[v];
        lv.target[v] = target[v];
        lv.grad[v] = grad[v];
        lv.count[v] = 3 * (int64_t)views[v].roi_w * views[v].roi_h;
        lv.blk_base[v + 1] = lv.blk_base[v] + gsp::loss_blocks(lv.count[v]);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = stage(ctx, "loss_l1", st, [&] { return gsp::launch_loss_l1(lv, loss, scratch, st); });
    if (e != hipSuccess) return hip_fail(e, "loss");
    return GSP_OK;
}

gsp_status gsp_loss_l1_noalloc(gsp_ctx *ctx, int32_t V, const gsp_view *views,
                               const float *const *pred, const float *const *target,
                               float *const *grad, float *loss, void *stream) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    if (!ctx->noalloc_scratch) return fail(GSP_EHIP, "fixed scratch of this device not set up");
    gsp::ViewsK vk;
    int64_t total_pix = 0;
    s = make_views(V, views, &vk, &total_pix);
    if (s != GSP_OK) return s;
    if (!pred || !target || !grad) return fail(GSP_EINVAL, "null pointer array");
    gsp::LossViewsK lv;
    std::memset(&lv, 0, sizeof lv);
    lv.V = V;
    lv.blk_base[0] = 0;
    for (int v = 0; v < V; v++) {
        if (!pred[v] || !target[v] || !grad[v])
            return fail(GSP_EINVAL, "null pred, target or grad of view %d", v);
        lv.pred[v] = pred[v];
        lv.target[v] = target[v];
        lv.grad[v] = grad[v];
        lv.count[v] = 3 * (int64_t)views[v].roi_w * views[v].roi_h;
        lv.blk_base[v + 1] = lv.blk_base[v] + gsp::loss_blocks(lv.count[v]);
    }
    const size_t need = (size_t)lv.blk_base[V] * sizeof(double);
    if (loss && need > gsp::kNoAllocScratchBytes)
        return fail(GSP_EINVAL,
                    "%lld loss blocks need %zu bytes of partial sums, more than the %zu of the "
                    "fixed scratch (at most %zu values over the views of a call)",
                    (long long)lv.blk_base[V], need, gsp::kNoAllocScratchBytes,
                    gsp::kNoAllocScratchBytes / sizeof(double) * gsp::kLossItems);
    // not bracketed by profiling events: this entry point creates nothing
    hipError_t e = gsp::launch_loss_l1(lv, loss, ctx->noalloc_scratch,
                                       static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "loss");
    return GSP_OK;
}

size_t gsp_loss_l1_scratch_bytes(int32_t V, const gsp_view *views) {
    int64_t blocks = 0;
    for (int v = 0; views && v < V; v++)
        blocks += gsp::loss_blocks(3 * (int64_t)views[v].roi_w * views[v].roi_h);
    return (size_t)(blocks > 0 ? blocks : 1) * sizeof(double);
}

gsp_status gsp_twist_apply(gsp_ctx *ctx, int32_t V, const float *tau, const float *poses,
                           float *out, void *stream) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    if (V < 1) return fail(GSP_EINVAL, "view count must be positive");
    if (!tau || !poses || !out) return fail(GSP_EINVAL, "null argument");
    hipError_t e = gsp::launch_twist_apply(V, tau, poses, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "twist apply");
    return GSP_OK;
}

gsp_status gsp_twist_chain(gsp_ctx *ctx, int32_t V, const float *tau, const float *dpose,
                           float *dtau, void *stream) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    if (V < 1) return fail(GSP_EINVAL, "view count must be positive");
    if (!tau || !dpose || !dtau) return fail(GSP_EINVAL, "null argument");
    if (dpose == dtau) return fail(GSP_EINVAL, "dtau may not alias dpose");
    hipError_t e = gsp::launch_twist_chain(V, tau, dpose, dtau, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "twist chain");
    return GSP_OK;
}

gsp_status gsp_pose_adam(gsp_ctx *ctx, int32_t V, float *poses, const float *dpose, float *m,
                         float *v, int32_t *steps, const gsp_adam_params *params,
                         const void *guard_workspace, void *stream) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    if (V < 1) return fail(GSP_EINVAL, "view count must be positive");
    if (!poses || !dpose || !m || !v || !steps || !params) return fail(GSP_EINVAL, "null argument");
    if (!(params->beta1 >= 0.f && params->beta1 < 1.f && params->beta2 >= 0.f &&
          params->beta2 < 1.f && params->eps > 0.f))
        return fail(GSP_EINVAL, "bad Adam hyper-parameters");
    if (params->parametrization != GSP_POSE_SE3 && params->parametrization != GSP_POSE_T_SO3)
        return fail(GSP_EINVAL, "unknown pose parametrization %d", params->parametrization);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = stage(ctx, "pose_adam", st, [&] {
        return gsp::launch_pose_adam(V, poses, dpose, m, v, steps, *params,
                                     static_cast<const uint32_t *>(guard_workspace), st);
    });
    if (e != hipSuccess) return hip_fail(e, "pose adam");
    return GSP_OK;
}

namespace {

// Normalised 11-tap Gaussian window of standard deviation 1.5, in double.
void ssim_window(float out[11]) {
    double w[11], sum = 0.0;
    for (int k = 0; k < 11; k++) {
        const double d = k - 5;
        w[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
        sum += w[k];
    }
    for (int k = 0; k < 11; k++) out[k] = (float)(w[k] / sum);
}

struct RgbLayout {
    int total_tiles;
    int64_t total_pix;
    size_t partial_bytes, total;
};

RgbLayout rgb_layout(int32_t V, const gsp_view *views) {
    RgbLayout L{0, 0, 0, 0};
    for (int v = 0; views && v < V; v++) {
        L.total_tiles += gsp::ssim_tiles(views[v].roi_w, views[v].roi_h);
        L.total_pix += (int64_t)views[v].roi_w * views[v].roi_h;
    }
    L.partial_bytes = align256((size_t)3 * (L.total_tiles > 0 ? L.total_tiles : 1) * sizeof(double2));
    L.total = L.partial_bytes + (size_t)9 * L.total_pix * sizeof(float);
    return L;
}

}  // namespace

gsp_status gsp_loss_rgb(gsp_ctx *ctx, int32_t V, const gsp_view *views, const float *const *pred,
                        const float *const *target, float *const *grad, float *loss, float beta,
                        void *scratch, size_t scratch_bytes, void *stream) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    gsp::ViewsK vk;
    int64_t total_pix = 0;
    s = make_views(V, views, &vk, &total_pix);
    if (s != GSP_OK) return s;
    if (!pred || !target || !grad) return fail(GSP_EINVAL, "null pointer array");
    if (!scratch) return fail(GSP_EINVAL, "null scratch");
    if (!(beta >= 0.f && beta <= 1.f)) return fail(GSP_EINVAL, "beta must lie in [0, 1]");
    const RgbLayout L = rgb_layout(V, views);
    if (scratch_bytes < L.total)
        return fail(GSP_ENOMEM, "scratch of %zu bytes is smaller than the %zu needed", scratch_bytes,
                    L.total);
    gsp::RgbViewsK a;
    std::memset(&a, 0, sizeof a);
    a.V = V;
    a.beta = beta;
    a.total_tiles = L.total_tiles;
    ssim_window(a.win);
    float *maps = reinterpret_cast<float *>(static_cast<char *>(scratch) + L.partial_bytes);
    int64_t pix = 0;
    for (int v = 0; v < V; v++) {
        if (!pred[v] || !target[v] || !grad[v])
            return fail(GSP_EINVAL, "null pred, target or grad of view %d", v);
        if (grad[v] == pred[v] || grad[v] == target[v])
            return fail(GSP_EINVAL, "grad of view %d aliases an input", v);
        a.pred[v] = pred[v];
        a.target[v] = target[v];
        a.grad[v] = grad[v];
        a.w[v] = views[v].roi_w;
        a.h[v] = views[v].roi_h;
        a.tiles_x[v] = (views[v].roi_w + 63) / 64;
        a.tile_base[v + 1] = a.tile_base[v] + gsp::ssim_tiles(views[v].roi_w, views[v].roi_h);
        a.gmap[v] = maps + 9 * pix;
        pix += (int64_t)views[v].roi_w * views[v].roi_h;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = stage(ctx, "loss_rgb", st, [&] {
        return gsp::launch_loss_rgb(a, loss, static_cast<double2 *>(scratch), st);
    });
    if (e != hipSuccess) return hip_fail(e, "rgb loss");
    return GSP_OK;
}

size_t gsp_loss_rgb_scratch_bytes(int32_t V, const gsp_view *views) {
    return rgb_layout(V, views).total;
}

gsp_status gsp_gaussian_adam(gsp_ctx *ctx, int64_t n, int32_t sh_degree,
                             const gsp_gaussian_params *params, const gsp_grads *grads, float *m,
                             float *v, int32_t step, const gsp_gaussian_adam_params *hp,
                             float *scales_out, float *opacities_out, float *aniso_loss,
                             void *scratch, const void *guard_workspace, void *stream) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(GSP_EINVAL, "bad Gaussian count");
    if (sh_degree < 0 || sh_degree > 3) return fail(GSP_EINVAL, "sh_degree must be 0..3");
    if (!params || !grads || !m || !v || !hp || !scales_out || !opacities_out)
        return fail(GSP_EINVAL, "null argument");
    if (!params->means || !params->log_scales || !params->quats || !params->logit_opacities ||
        !params->sh)
        return fail(GSP_EINVAL, "null parameter array");
    if (!grads->means || !grads->scales || !grads->quats || !grads->opacities || !grads->sh)
        return fail(GSP_EINVAL, "every Gaussian gradient is needed");
    if (step < 1) return fail(GSP_EINVAL, "step counts from 1");
    if (!(hp->beta1 >= 0.0 && hp->beta1 < 1.0 && hp->beta2 >= 0.0 && hp->beta2 < 1.0 &&
          hp->eps > 0.0 && hp->total_steps >= 1 && hp->lr_means_start > 0.0 &&
          hp->lr_means_end > 0.0 && hp->lr_sh_dc >= 0.0 && hp->lr_sh_rest >= 0.0 &&
          hp->lr_opacities >= 0.0 && hp->lr_scales >= 0.0 && hp->lr_quats >= 0.0 &&
          hp->aniso_r > 0.0 && hp->aniso_weight >= 0.0))
        return fail(GSP_EINVAL, "bad Adam hyper-parameters");
    if (aniso_loss && !scratch) return fail(GSP_EINVAL, "aniso_loss requires scratch memory");
    const int S = (sh_degree + 1) * (sh_degree + 1);
    gsp::GaussAdamK a;
    std::memset(&a, 0, sizeof a);
    a.means = params->means;
    a.log_scales = params->log_scales;
    a.quats = params->quats;
    a.logits = params->logit_opacities;
    a.sh = params->sh;
    a.g_means = grads->means;
    a.g_scales = grads->scales;
    a.g_quats = grads->quats;
    a.g_opacities = grads->opacities;
    a.g_sh = grads->sh;
    a.m = m;
    a.v = v;
    a.scales_out = scales_out;
    a.opacities_out = opacities_out;
    a.partial = aniso_loss ? static_cast<double *>(scratch) : nullptr;
    a.guard = static_cast<const uint32_t *>(guard_workspace);
    a.n = n;
    a.S = S;
    a.items[0] = 3 * n;
    a.items[1] = a.items[0] + n;
    a.items[2] = a.items[1] + 4 * n;
    a.items[3] = a.items[2] + n;
    a.items[4] = a.items[3] + 3 * (int64_t)S * n;
    a.moff[0] = 0;
    a.moff[1] = 3 * n;
    a.moff[2] = 6 * n;
    a.moff[3] = 10 * n;
    a.moff[4] = 11 * n;
    double t = 0.0;
    if (hp->total_steps > 1)
        t = (double)std::min(step - 1, hp->total_steps - 1) / (double)(hp->total_steps - 1);
    a.lr_means = std::exp(std::log(hp->lr_means_start) * (1.0 - t) + std::log(hp->lr_means_end) * t);
    a.lr_scales = hp->lr_scales;
    a.lr_quats = hp->lr_quats;
    a.lr_opacities = hp->lr_opacities;
    a.lr_sh_dc = hp->lr_sh_dc;
    a.lr_sh_rest = hp->lr_sh_rest;
    a.b1 = hp->beta1;
    a.b2 = hp->beta2;
    a.c1 = 1.0 - std::pow(hp->beta1, (double)step);
    a.c2 = 1.0 - std::pow(hp->beta2, (double)step);
    a.eps = hp->eps;
    a.aniso_r = hp->aniso_r;
    a.aniso_w = hp->aniso_weight;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = stage(ctx, "gaussian_adam", st, [&] {
        return gsp::launch_gauss_adam(a, aniso_loss, st);
    });
    if (e != hipSuccess) return hip_fail(e, "gaussian adam");
    return GSP_OK;
}

gsp_status gsp_unproject_count(const gsp_view *view, int32_t stride, int64_t *n) {
    gsp::ViewsK vk;
    int64_t total_pix = 0;
    gsp_status s = make_views(1, view, &vk, &total_pix);
    if (s != GSP_OK) return s;
    if (stride < 1) return fail(GSP_EINVAL, "stride must be positive");
    if (!n) return fail(GSP_EINVAL, "null output");
    *n = (int64_t)((view->roi_w + stride - 1) / stride) * ((view->roi_h + stride - 1) / stride);
    return GSP_OK;
}

size_t gsp_unproject_scratch_bytes(const gsp_view *view, int32_t stride) {
    int64_t n = 0;
    if (gsp_unproject_count(view, stride, &n) != GSP_OK) return 0;
    return (size_t)(n > 0 ? n : 1) * sizeof(float4);
}

gsp_status gsp_unproject(gsp_ctx *ctx, const gsp_view *view, const float *depth,
                         const float *image, int32_t stride, float opacity, int32_t sh_degree,
                         const gsp_gaussian_params *out, void *scratch, size_t scratch_bytes,
                         void *stream) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    int64_t n = 0;
    s = gsp_unproject_count(view, stride, &n);
    if (s != GSP_OK) return s;
    if (n > gsp::kMaxUnprojectPoints)
        return fail(GSP_EINVAL, "%lld points exceed the %d the brute-force neighbour search takes; "
                    "use a larger stride", (long long)n, gsp::kMaxUnprojectPoints);
    if (!depth || !image || !out || !scratch) return fail(GSP_EINVAL, "null argument");
    if (!out->means || !out->log_scales || !out->quats || !out->logit_opacities || !out->sh)
        return fail(GSP_EINVAL, "null parameter array");
    if (sh_degree < 0 || sh_degree > 3) return fail(GSP_EINVAL, "sh_degree must be 0..3");
    if (!(opacity > 0.f && opacity < 1.f)) return fail(GSP_EINVAL, "opacity must lie in (0, 1)");
    if (scratch_bytes < gsp_unproject_scratch_bytes(view, stride))
        return fail(GSP_ENOMEM, "scratch too small");
    gsp::UnprojK a;
    std::memset(&a, 0, sizeof a);
    a.depth = depth;
    a.image = image;
    a.w = view->roi_w;
    a.h = view->roi_h;
    a.stride = stride;
    a.nx = (view->roi_w + stride - 1) / stride;
    a.ny = (view->roi_h + stride - 1) / stride;
    a.S = (sh_degree + 1) * (sh_degree + 1);
    a.roi_x = view->roi_x;
    a.roi_y = view->roi_y;
    a.fx = view->fx;
    a.fy = view->fy;
    a.cx = view->cx;
    a.cy = view->cy;
    a.logit = (float)std::log((double)opacity / (1.0 - (double)opacity));
    a.means = out->means;
    a.log_scales = out->log_scales;
    a.quats = out->quats;
    a.logits = out->logit_opacities;
    a.sh = out->sh;
    a.pts = static_cast<float4 *>(scratch);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = stage(ctx, "unproject", st, [&] { return gsp::launch_unproject(a, st); });
    if (e != hipSuccess) return hip_fail(e, "unproject");
    return GSP_OK;
}

gsp_status gsp_loss_masked_l1(gsp_ctx *ctx, int32_t V, const gsp_view *views,
                              const float *const *pred, const float *const *target,
                              const float *const *alpha, float *const *grad, float *loss,
                              void *scratch, void *stream) {
    gsp_status s = check_device(ctx);
    if (s != GSP_OK) return s;
    gsp::ViewsK vk;
    int64_t total_pix = 0;
    s = make_views(V, views, &vk, &total_pix);
    if (s != GSP_OK) return s;
    if (!pred || !target || !alpha || !grad) return fail(GSP_EINVAL, "null pointer array");
    if (loss && !scratch) return fail(GSP_EINVAL, "loss requires scratch memory");
    gsp::MaskViewsK a;
    std::memset(&a, 0, sizeof a);
    a.V = V;
    for (int v = 0; v < V; v++) {
        if (!pred[v] || !target[v] || !alpha[v] || !grad[v])
            return fail(GSP_EINVAL, "null pred, target, alpha or grad of view %d", v);
        a.pred[v] = pred[v];
        a.target[v] = target[v];
        a.alpha[v] = alpha[v];
        a.grad[v] = grad[v];
        a.pix[v] = (int64_t)views[v].roi_w * views[v].roi_h;
        a.blk_base[v + 1] = a.blk_base[v] + gsp::masked_blocks(3 * a.pix[v]);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = stage(ctx, "loss_masked_l1", st,
                         [&] { return gsp::launch_masked_l1(a, loss, scratch, st); });
    if (e != hipSuccess) return hip_fail(e, "masked loss");
    return GSP_OK;
}

size_t gsp_loss_masked_l1_scratch_bytes(int32_t V, const gsp_view *views) {
    int64_t blocks = 0;
    for (int v = 0; views && v < V; v++)
        blocks += gsp::masked_blocks(3 * (int64_t)views[v].roi_w * views[v].roi_h);
    return (size_t)(blocks > 0 ? blocks : 1) * sizeof(double);
}

size_t gsp_gaussian_adam_scratch_bytes(int64_t n) {
    const int64_t p = gsp::gauss_adam_partials(n);
    return (size_t)(p > 0 ? p : 1) * sizeof(double);
}

}  // extern "C"
