// preprocess.hip -- projection of every Gaussian into every view of a call,
// and duplication of each projected splat into its tile instances.
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
        }
    }
}

// Per-block sums of the tile counts of the view-Gaussians in index order
// (kScanItems per block, kScanPerThread consecutive ones per thread), and
// the number of them with at least one instance.
__global__ __launch_bounds__(kPreprocessBlock) void k_blocksums(const uint32_t *tiles,
                                                                unsigned long long *bs,
                                                                uint32_t *bvis, int vn) {
    __shared__ unsigned long long red[kPreprocessBlock / kWave];
    const int k0 = blockIdx.x * kScanItems + kScanPerThread * threadIdx.x;
    unsigned long long cnt = 0, vis = 0;
#pragma unroll
    for (int j = 0; j < kScanPerThread; j++) {
        const uint32_t c = k0 + j < vn ? tiles[k0 + j] : 0u;
        cnt += c;
        vis += c > 0 ? 1ull : 0ull;
    }
    const unsigned long long s = block_sum<unsigned long long, kPreprocessBlock>(cnt, red);
    const unsigned long long v = block_sum<unsigned long long, kPreprocessBlock>(vis, red);
    if (threadIdx.x == 0) {
        bs[blockIdx.x] = s;
        bvis[blockIdx.x] = (uint32_t)v;
    }
}

struct DupArgs {
    const uint2 *rect;
    const uint32_t *tiles;
    uint32_t *offsets;             // [vn + 1] first emission position of each view-Gaussian, then M
    uint32_t *vis;                 // [vn] the view-Gaussians with instances, in index order
    uint32_t *offv;                // [vn + 1] first emission position of each of those, then M
    uint2 *wstart;                 // [windows + 1] first view-Gaussian of each work window and its first slot
    uint32_t *pstart;              // [emission blocks + 1] rank in vis owning each block's start
    const unsigned long long *blocksum;  // [nblk] per-block tile counts in index order
    const uint32_t *blockvis;      // [nblk] per-block counts of view-Gaussians with instances
    uint32_t *counters;
    uint32_t *keys;
    uint32_t *vals;
    uint32_t *hist;                // [kSortBins][eblk] low-digit counts of each emission block
    uint32_t mask0;                // low digit of the instance sort's first pass
    uint32_t *ranges;              // [2 * total_tiles], cleared here
    uint8_t *slot_flags;           // [cap][kSplitBwd], cleared here for positions < M
    unsigned long long cap;
    int vn, nblk, eblk, total_tiles;
    int sort_items;                // instance positions per emission (and sort) block
    int vbits;                     // > 0: emit packed (tile << vbits | value) into keys only
};

// Exclusive offsets of the splats' instance runs in index order (the
// emission positions, which are also the backward's gradient slots), the
// list of the splats with instances (vis, with their offsets offv), the work
// windows and the emission blocks.  Each block first sums the block sums
// before it (and all of them, for M and the overflow flag; block 0 writes
// the counters).  Splat k's entry sits at position h = k + offsets[k] of the
// sequence (splat, its instances, next splat, ...), the next at h + 1 + cnt;
// window b starts at the first splat whose entry is at or after b * kWindow.
// Emission block p covers instance positions [p, p + 1) * items (items =
// the sort's block size) and starts at the splat of vis whose run holds
// position p * items; entry ceil(M / items) is the last of vis.  The
// emission works on vis, not on all splats: the positions of one block then
// belong to at most items + 1 splats, however many culled splats lie
// between them.
__global__ __launch_bounds__(kPreprocessBlock) void k_offsets(DupArgs a) {
    __shared__ unsigned long long scratch[kPreprocessBlock / kWave];
    const int t = threadIdx.x;
    unsigned long long before = 0, all = 0, vbefore = 0;
    for (int j = t; j < a.nblk; j += kPreprocessBlock) {
        const unsigned long long x = a.blocksum[j];
        all += x;
        if (j < (int)blockIdx.x) {
            before += x;
            vbefore += a.blockvis[j];
        }
    }
    before = block_sum<unsigned long long, kPreprocessBlock>(before, scratch);
    all = block_sum<unsigned long long, kPreprocessBlock>(all, scratch);
    vbefore = block_sum<unsigned long long, kPreprocessBlock>(vbefore, scratch);
    const bool ovf = all > a.cap;
    if (blockIdx.x == 0 && t == 0) {
        a.counters[kCntMLo] = (uint32_t)(all & 0xffffffffull);
        a.counters[kCntMHi] = (uint32_t)(all >> 32);
        a.counters[kCntOverflow] = ovf ? 1u : 0u;
        a.counters[kCntMEff] = ovf ? 0u : (uint32_t)all;
        if (ovf) a.counters[kCntSticky] = 1u;
        if (a.vn == 0) a.counters[kCntWin] = 0u;
    }
    const int k0 = blockIdx.x * kScanItems + kScanPerThread * t;
    uint32_t cnt[kScanPerThread];
    unsigned long long local = 0, vlocal = 0;
#pragma unroll
    for (int j = 0; j < kScanPerThread; j++) {
        cnt[j] = k0 + j < a.vn ? a.tiles[k0 + j] : 0u;
        local += cnt[j];
        vlocal += cnt[j] > 0 ? 1ull : 0ull;
    }
    unsigned long long total;
    unsigned long long excl =
        block_exclusive_scan<unsigned long long, kPreprocessBlock>(local, scratch, &total) + before;
    unsigned long long vexcl =
        block_exclusive_scan<unsigned long long, kPreprocessBlock>(vlocal, scratch, &total) + vbefore;
    if (ovf) return;
#pragma unroll
    for (int j = 0; j < kScanPerThread; j++) {
        const int k = k0 + j;
        if (k >= a.vn) break;
        a.offsets[k] = (uint32_t)excl;
        const unsigned long long h = (unsigned long long)k + excl, h1 = h + 1 + cnt[j];
        const unsigned long long e1 = excl + cnt[j];
        if (k == 0) a.wstart[0] = make_uint2(0u, 0u);
        for (unsigned long long b = h / kWindow + 1; b * kWindow <= h1; b++)
            a.wstart[b] = make_uint2((uint32_t)k + 1, (uint32_t)e1);
        if (cnt[j] > 0) {
            a.vis[vexcl] = (uint32_t)k;
            a.offv[vexcl] = (uint32_t)excl;
            const unsigned long long items = (unsigned long long)a.sort_items;
            for (unsigned long long p = (excl + items - 1) / items; p * items < e1; p++)
                a.pstart[p] = (uint32_t)vexcl;
            if (e1 == all) {
                a.pstart[(all + items - 1) / items] = (uint32_t)vexcl;
                a.offv[vexcl + 1] = (uint32_t)all;
            }
            vexcl++;
        }
        if (k == a.vn - 1) {
            const unsigned long long nwin = (h1 + kWindow - 1) / kWindow;
            if (nwin * kWindow > h1) a.wstart[nwin] = make_uint2((uint32_t)a.vn, (uint32_t)e1);
            a.offsets[a.vn] = (uint32_t)e1;
            a.counters[kCntWin] = (uint32_t)nwin;
        }
        excl = e1;
    }
}

#ifndef GSP_EMIT_THREADS
#define GSP_EMIT_THREADS 256
#endif
constexpr int kEmitThreads = GSP_EMIT_THREADS;
static_assert(kEmitThreads >= kSortBins && kEmitThreads <= 1024 && kEmitThreads % kWave == 0,
              "emission block size");

// Emits one (tile, view * n + i) pair per tile of each splat's rect, rows
// outer and columns inner, at the splat's offset; a stable sort of these
// pairs by tile then yields every tile's list in index order, which the
// per-tile depth sort turns into (depth, index) order.
// Block p writes instance positions [p, p + 1) * ITEMS, which are the
// keys of block p of the first pass of that sort, so it also writes their
// low-digit histogram (zeros past M); each thread finds the splat owning a
// position by binary search over the block's offsets in LDS.  The blocks
// also clear the tile ranges and the backward's slot flags of their
// positions, which the later stages of this forward and of its backward
// fill in.
template <int ITEMS>
__global__ __launch_bounds__(kEmitThreads) void k_emit(DupArgs a, ViewsK views, int n) {
    static_assert(kEmitThreads % kSortBins == 0, "whole histograms per block");
    constexpr int kMaxSplats = ITEMS + 1;
    __shared__ uint32_t s_off[kMaxSplats + 1];
    __shared__ uint32_t s_idx[kMaxSplats];
    __shared__ uint2 s_rect[kMaxSplats];
    __shared__ uint32_t s_hist[kSortBins];
    const int b = blockIdx.x, t = threadIdx.x;
    for (int i = b * kEmitThreads + t; i < 2 * a.total_tiles; i += gridDim.x * kEmitThreads)
        a.ranges[i] = 0u;
    if (t < kSortBins) s_hist[t] = 0u;
    // pstart has eblk + 1 entries; they are read before M is known (those of
    // blocks past M are stale and unused)
    const uint32_t kb = a.pstart[b], kn = a.pstart[b + 1];
    const uint32_t M = a.counters[kCntMEff];
    const uint32_t p0 = (uint32_t)b * ITEMS;
    if (p0 < M) {
        const uint32_t p1 = min(p0 + (uint32_t)ITEMS, M);
        const int nk = min((int)(kn + 1 - kb), kMaxSplats);
        for (int j = t; j < nk; j += kEmitThreads) {
            const uint32_t idx = a.vis[kb + j];
            s_off[j] = a.offv[kb + j];
            s_idx[j] = idx;
            s_rect[j] = a.rect[idx];
        }
        if (t == 0) s_off[nk] = a.offv[kb + nk];
        __syncthreads();
        // Each thread emits kPer consecutive positions: a binary search for
        // the first, then a walk along the splats' tiles (rows outer,
        // columns inner), with no division per position.
        constexpr int kPer = ITEMS / kEmitThreads;
        static_assert(ITEMS % kEmitThreads == 0, "whole runs of positions per thread");
        const uint32_t e0 = p0 + (uint32_t)t * kPer;
        if (e0 < p1) {
            // largest j with s_off[j] <= e0; s_off[0] <= p0 <= e0 < p1 <= s_off[nk]
            int lo = 0, hi = nk;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_off[mid] <= e0) lo = mid; else hi = mid;
            }
            uint32_t next = 0, idx = 0, w = 1, x0 = 0, y0 = 0, tbase = 0, gw = 0, tx = 0, ty = 0;
            // the splat at entry lo, and the tile of position e in it
            auto enter = [&](uint32_t e) {
                next = s_off[lo + 1];
                const uint2 r = s_rect[lo];
                x0 = r.x & 0xffff;
                y0 = r.x >> 16;
                w = (r.y & 0xffff) - x0;
                idx = s_idx[lo];
                const ViewK &vw = views.v[idx / (uint32_t)n];
                tbase = (uint32_t)vw.tile_base;
                gw = (uint32_t)vw.gw;
                const uint32_t local = e - s_off[lo];
                ty = local / w;
                tx = local - ty * w;
            };
            enter(e0);
            const int cnt = (int)min((uint32_t)kPer, p1 - e0);
            uint32_t kk[kPer], vv[kPer];
#pragma unroll
            for (int q = 0; q < kPer; q++) {
                if (q < cnt) {
                    const uint32_t e = e0 + (uint32_t)q;
                    if (e >= next) {   // a later splat: the last one whose offset is <= e
                        do lo++;
                        while (s_off[lo + 1] <= e);
                        enter(e);
                    }
                    const uint32_t key = tbase + (y0 + ty) * gw + x0 + tx;
                    kk[q] = a.vbits > 0 ? (key << a.vbits) | idx : key;
                    vv[q] = idx;
                    atomicAdd(&s_hist[key & a.mask0], 1u);
                    if (++tx == w) {
                        tx = 0;
                        ty++;
                    }
                }
            }
            // e0 is a multiple of kPer and the regions are 256-byte aligned,
            // so a full run is stored as 16-byte vectors
            static_assert(kPer % 4 == 0, "vector stores of a run");
            if (cnt == kPer) {
#pragma unroll
                for (int q = 0; q < kPer; q += 4)
                    *reinterpret_cast<uint4 *>(a.keys + e0 + q) = make_uint4(kk[q], kk[q + 1], kk[q + 2], kk[q + 3]);
                if (a.vbits == 0) {
#pragma unroll
                    for (int q = 0; q < kPer; q += 4)
                        *reinterpret_cast<uint4 *>(a.vals + e0 + q) = make_uint4(vv[q], vv[q + 1], vv[q + 2], vv[q + 3]);
                }
#pragma unroll
                for (int q = 0; q < kSplitBwd * kPer / 4; q++)
                    reinterpret_cast<uint32_t *>(a.slot_flags + (size_t)kSplitBwd * e0)[q] = 0u;
            } else {
                for (int q = 0; q < cnt; q++) {
                    a.keys[e0 + q] = kk[q];
                    if (a.vbits == 0) a.vals[e0 + q] = vv[q];
                    for (int k = 0; k < kSplitBwd; k++) a.slot_flags[(size_t)kSplitBwd * (e0 + q) + k] = 0;
                }
            }
        }
    }
    __syncthreads();
    if ((uint32_t)t <= a.mask0) a.hist[(size_t)t * a.eblk + b] = s_hist[t];   // rows of used digits
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
    DupArgs a;
    a.rect = region<uint2>(ws, L.rect);
    a.tiles = region<uint32_t>(ws, L.tiles);
    a.offsets = region<uint32_t>(ws, L.offsets);
    a.vis = region<uint32_t>(ws, L.vis);
    a.offv = region<uint32_t>(ws, L.offv);
    a.blockvis = region<uint32_t>(ws, L.blockvis);
    a.wstart = region<uint2>(ws, L.wstart);
    a.pstart = region<uint32_t>(ws, L.pstart);
    a.blocksum = region<unsigned long long>(ws, L.blocksum);
    a.counters = region<uint32_t>(ws, L.counters);
    a.keys = region<uint32_t>(ws, L.keys0);
    a.vals = region<uint32_t>(ws, L.vals0);
    a.hist = region<uint32_t>(ws, L.hist);
    a.mask0 = (1u << digit_bits(L.tile_bits)) - 1u;
    a.ranges = region<uint32_t>(ws, L.ranges);
    a.slot_flags = region<uint8_t>(ws, L.slot_flags);
    a.cap = (unsigned long long)L.cap;
    a.vn = (int)L.vn;
    a.nblk = L.nblk_scan;
    a.eblk = L.nblk_emit;
    a.total_tiles = L.total_tiles;
    a.sort_items = L.sort_items;
    a.vbits = L.sort_vbits;
    if (a.vn > 0) {
        hipLaunchKernelGGL(k_blocksums, dim3(L.nblk_scan), dim3(kPreprocessBlock), 0, s, a.tiles,
                           region<unsigned long long>(ws, L.blocksum),
                           region<uint32_t>(ws, L.blockvis), a.vn);
    }
    hipLaunchKernelGGL(k_offsets, dim3(L.nblk_scan > 0 ? L.nblk_scan : 1), dim3(kPreprocessBlock),
                       0, s, a);
    if (L.sort_items == kSortThreads * kSortRoundsLarge)
        hipLaunchKernelGGL(k_emit<kSortThreads * kSortRoundsLarge>, dim3(L.nblk_emit),
                           dim3(kEmitThreads), 0, s, a, views, (int)L.n);
    else
        hipLaunchKernelGGL(k_emit<kSortThreads * kSortRoundsSmall>, dim3(L.nblk_emit),
                           dim3(kEmitThreads), 0, s, a, views, (int)L.n);
    return hipGetLastError();
}

}  // namespace gsp
