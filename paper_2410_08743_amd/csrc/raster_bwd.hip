// raster_bwd.hip -- backward of the compositing of Eq. (3)-(4).
//
// For the blended entries i of a pixel, with upstream G = dL/dC and T_i the
// transmittance in front of i:
//   dL/dc_i     = G alpha_i T_i
//   dL/dalpha_i = T_i G . (c_i - S_i),  S_i = colour behind i seen through i,
//   S_last = bg,  S_{i-1} = alpha_i c_i + (1 - alpha_i) S_i
// and through alpha = o exp(power) (no gradient when clamped at 0.99):
//   dL/dpower = dL/dalpha alpha,  dL/do = dL/dpower / o,
//   dpower/du = -(A dx + B dy), dpower/dv = -(C dy + B dx),
//   dpower/dA = -dx^2/2, dpower/dB = -dx dy, dpower/dC = -dy^2/2.
//
// MI355X design: nothing per pixel is stored by the forward beyond T_final,
// the contributor count and, for lists that are cut, the final colour and
// (T, accumulated colour) at every cut.  The work items are (tile, chunk)
// pairs, so that no workgroup walks more than a chunk of a list that is cut
// (the longest lists would otherwise run alone at the end of the launch);
// kSplit wavefronts per item (one by default, the whole tile), each a strip
// of rows, walk the chunk back to front from the largest contributor count
// of their pixels inside it,
// recovering T_i = T_{i+1} / (1 - alpha_i) with the forward's exact
// evaluation, and skip (per lane-parallel bound, as in the forward) the
// entries that reach 1/255 nowhere in their rows.  Each lane
// sums its pixels in registers; the nine sums are reduced over the 64 lanes
// in two steps: v_permlane32_swap and v_permlane16_swap leave each as 16
// partial sums in one row of lanes (16 VALU operations for the nine), which
// wait in LDS; every kPend entries, 63 lanes each add up the 16 partials of
// one (entry, component) in a fixed order and store it into the strip's part
// of the instance's own slot (its position in emission order), flagging it
// written.  No atomics: the per-splat sum over its slots happens later in a
// fixed order, so gradients are bit-reproducible.
#include <cstring>
#include <type_traits>

#include "block_ops.h"
#include "raster_common.h"

namespace gsp {

constexpr int kSplit = kSplitBwd;
constexpr int kPixPerLane = 4 / kSplit;   // pixels per lane, one column

struct BwdArgs {
    const uint32_t *items;   // work items tile * kMaxChunks + chunk, longest first
    const uint32_t *counters;
    const float4 *ckpt;
    const float *cfinal;
    int total_pix;
    const uint2 *ranges;
    const uint32_t *vals;
    const float4 *geom;
    const float4 *color;
    const uint2 *rect;
    const uint32_t *offsets;
    const float *tfinal;
    const uint32_t *ncontrib;
    float *slots;          // [cap][kSplit][9]
    uint8_t *slot_flags;   // [cap][kSplit]: 1 where this kernel wrote the slot
    // stored-list variant only
    const uint32_t *order;     // tiles, longest list first
    const uint32_t *loff;      // [total_pix + 1] first pair of each pixel
    const PairRec *pairs;
    const uint32_t *lhdr;      // list header (overflow flag)
    int total_tiles;
};

constexpr uint32_t kNoSlot = 0xffffffffu;

#ifndef GSP_BWD_UNROLL
#define GSP_BWD_UNROLL 2
#endif
constexpr int kBwdUnroll = GSP_BWD_UNROLL;   // entries whose LDS records are read together
// Entries whose row partials wait in LDS before a flush (at most 7: nine
// lanes per entry in the flush).
#ifndef GSP_BWD_PEND
#define GSP_BWD_PEND 7
#endif
static_assert(GSP_BWD_PEND >= 1 && 9 * GSP_BWD_PEND <= 64, "one flush lane per (entry, component)");
// 1: each group's records are read while the group before it is processed
#ifndef GSP_BWD_PREFETCH
#define GSP_BWD_PREFETCH 0
#endif

// Slot of the instance of splat `id` in tile (tx, ty): its emission position.
__device__ __forceinline__ uint32_t slot_of(const BwdArgs &a, uint32_t id, int tx, int ty) {
    const uint2 r = a.rect[id];
    const int x0 = r.x & 0xffff, y0 = r.x >> 16, x1 = r.y & 0xffff;
    return a.offsets[id] + (uint32_t)((ty - y0) * (x1 - x0) + (tx - x0));
}

#ifndef GSP_BWD_WAVES
#define GSP_BWD_WAVES 4
#endif
// Pixel with no stored pair left, and the list position of padding records
// (never a pixel's next pair; below every pixel's count as a signed int, and
// the padding's empty band mask skips it in either walk).
constexpr uint32_t kNoPos = 0xffffffffu;
constexpr uint32_t kPadPos = 0xfffffffeu;

// STORED = false: the recomputing backward over (tile, chunk) work items.
// STORED = true: one workgroup per whole tile; each pixel's blended entries,
// with their alpha and the transmittance in front of them, come from the
// pair records the forward stored (GSP_STORE_LISTS); the walk, the
// culling, the gradient formulas and the reduction are the same.
// OPA = false (no opacity gradient wanted, e.g. a pose-only solve): the
// wave reduces eight sums per entry instead of nine (the opacity sum, which
// only the opacity gradient needs, is left out) and the slot's opacity
// component is written as zero.
template <bool STORED, bool OPA>
__global__ __launch_bounds__(kRasterThreads) __attribute__((amdgpu_waves_per_eu(GSP_BWD_WAVES))) void k_raster_bwd(BwdArgs a, ViewsK views) {
    __shared__ StagedA sA[kBatch];
    __shared__ StagedB sB[kBatch];
    __shared__ StagedC sC[kBatch];
    __shared__ uint32_t sM[kBatch];   // bands the entry may reach (band_mask)
    // Row partials of the nine sums of up to kPend entries (wave_sum9_rows),
    // register-major, rows kRowStride floats apart so that the 63 lanes of a
    // flush, each reading its own row, spread over the banks; and the slot
    // and 1/o of each pending entry.
    constexpr int kPend = GSP_BWD_PEND;
    constexpr int kRowStride = 17;
    constexpr int kRegStride = 4 * kRowStride;
    constexpr int kEntryStride = 3 * kRegStride;
    __shared__ float sP[kPend * kEntryStride];
    __shared__ uint32_t sPs[kPend];
    __shared__ float sPi[kPend];
    int rank, part;
    part_of_block<kSplit>(blockIdx.x, rank, part);
    uint32_t item;
    if (STORED) {
        if (rank >= a.total_tiles || a.lhdr[kListOverflow]) return;
        item = a.order[rank] * kMaxChunks;   // chunk 0 of an uncut walk
    } else {
        if ((uint32_t)rank >= a.counters[kCntItems]) return;
        item = a.items[rank];
    }
    const int tile = (int)(item / kMaxChunks), chunk = (int)(item % kMaxChunks);
    const ViewK &vw = views.v[view_of_tile(views, tile)];
    const int lt = tile - vw.tile_base;
    const int tx = lt % vw.gw, ty = lt / vw.gw;
    const int px0 = vw.roi_x + kTile * tx, py0 = vw.roi_y + kTile * ty;
    const int lane = threadIdx.x;
    const int lx = lane & 15, ly = lane >> 4;
    const int rx = kTile * tx + lx;
    const int P = vw.roi_w * vw.roi_h;
    const int row0 = part * (kTile / kSplit);   // first tile row of this part
    float *const pslots = a.slots + 9 * part;   // this part's slot of each instance
    uint8_t *const pflags = a.slot_flags + part;

    // In a flush, lane k < 9 kPend sums component pc of pending entry pe,
    // whose row partials start at poff within the entry's area; pscale is
    // the component's scale (see the base-2 conic of raster_common.h; the
    // opacity's 1/o comes with the entry).
    const int pe = lane / 9, pc = lane % 9;
    const int pc8 = pc < 5 ? pc : pc - 1;   // position among the eight sums (pc != 5)
    const int poff = OPA ? ((pc == 8 ? 2 : pc >> 2) * 4 + sum9_row(pc)) * kRowStride
                         : ((pc8 >> 2) * 4 + sum9_row(pc8)) * kRowStride;
    const float pscale = pc == 0 || pc == 1 ? kLn2 : pc == 2 || pc == 4 ? -0.5f : pc == 3 ? -1.f : 1.f;
    int npend = 0;
    auto flush = [&]() {
        __syncthreads();   // one wavefront: orders the stashing stores before these loads
        if (lane < 9 * npend) {
            const float *src = sP + pe * kEntryStride + poff;
            float t[8];
#pragma unroll
            for (int i = 0; i < 8; i++) t[i] = src[i] + src[8 + i];
#pragma unroll
            for (int i = 0; i < 4; i++) t[i] += t[4 + i];
            const float sum = (t[0] + t[2]) + (t[1] + t[3]);
            const uint32_t slot = sPs[pe];
            if (slot != kNoSlot) {
                const float f = pc == 5 ? sPi[pe] : pscale;
                pslots[9 * kSplit * (size_t)slot + pc] = OPA || pc != 5 ? sum * f : 0.f;
                if (pc == 0) pflags[kSplit * (size_t)slot] = 1;
            }
        }
        __syncthreads();   // before the next entries overwrite the area
        npend = 0;
    };

    // GS = G . S: the upstream gradient dotted with the colour behind the
    // current splat, which is all that dL/dalpha needs of S.
    // This chunk holds list positions [clo, chi).  A pixel that composited
    // past chi starts at chi from the state the forward recorded at that
    // cut; the others start from their final state at their contributor
    // count, as in an unsplit walk.
    const uint2 rg = a.ranges[tile];
    const int len = (int)(rg.y - rg.x);
    const int nch = STORED ? 1 : chunks_of(len);
    const int clo = chunk * kChunk, chi = chunk == nch - 1 ? len : clo + kChunk;
    const float4 *const ck =
        chunk < nch - 1 ? a.ckpt + (size_t)((rg.x + (uint32_t)chi) / kChunk) * (kTile * kTile)
                        : nullptr;
    float T[kPixPerLane], G[kPixPerLane][3], GS[kPixPerLane], fy[kPixPerLane];
    int last[kPixPerLane];
    // stored lists: the pixel's next pair back to front (position, alpha, T)
    // and its index; pbase is the pixel's first pair
    uint32_t npos[kPixPerLane], pidx[kPixPerLane], pbase[kPixPerLane];
    float nal[kPixPerLane];
    int maxlast = 0;
#pragma unroll
    for (int q = 0; q < kPixPerLane; q++) {
        const int ryl = row0 + ly + 4 * q;
        const int ry = kTile * ty + ryl;
        const bool in = rx < vw.roi_w && ry < vw.roi_h;
        const size_t pix = (size_t)ry * vw.roi_w + rx;
        fy[q] = (float)ryl;
        if (STORED) {
            npos[q] = kNoPos;
            nal[q] = 0.f;
            T[q] = 1.f;
            pbase[q] = in ? a.loff[vw.pix_base + pix] : 0u;
            pidx[q] = in ? a.loff[vw.pix_base + pix + 1] : 0u;   // one past the last pair
            last[q] = 0;
            if (pidx[q] > pbase[q]) {
                pidx[q]--;
                const PairRec r = a.pairs[pidx[q]];
                npos[q] = r.pos;
                nal[q] = r.alpha;
                T[q] = r.T;
                last[q] = (int)r.pos + 1;
            }
        } else {
            T[q] = in ? a.tfinal[vw.pix_base + pix] : 1.f;
            last[q] = in ? (int)a.ncontrib[vw.pix_base + pix] : 0;
        }
        const float *dl = vw.dl;
        G[q][0] = in ? dl[pix] : 0.f;
        G[q][1] = in ? dl[(size_t)P + pix] : 0.f;
        G[q][2] = in ? dl[2 * (size_t)P + pix] : 0.f;
        float S0 = vw.bg[0], S1 = vw.bg[1], S2 = vw.bg[2];
        if (!STORED && last[q] > chi) {   // only when this chunk ends at a cut
            // final colour = colour in front of the cut + T_cut * colour behind it
            const float4 c = ck[ryl * kTile + lx];
            const size_t pf = (size_t)vw.pix_base + pix;
            const float inv = 1.f / c.x;
            T[q] = c.x;
            S0 = (a.cfinal[pf] - c.y) * inv;
            S1 = (a.cfinal[(size_t)a.total_pix + pf] - c.z) * inv;
            S2 = (a.cfinal[2 * (size_t)a.total_pix + pf] - c.w) * inv;
            last[q] = chi;
        }
        GS[q] = G[q][0] * S0 + G[q][1] * S1 + G[q][2] * S2;
        maxlast = max(maxlast, last[q]);
    }
    maxlast = wave_max(maxlast);
    // largest contributor count of each band: an entry at or past it has no
    // candidate pixel in the band
    int blast[kPixPerLane];
#pragma unroll
    for (int q = 0; q < kPixPerLane; q++) blast[q] = __builtin_amdgcn_readfirstlane(wave_max(last[q]));
    const float fxl = (float)lx;

    // batches of 64 entries ending at hi, walked back to front; positions
    // below clo are absent.  Records are gathered one batch ahead.
    float4 g0, g1, gc;
    uint32_t gslot;
    auto gather = [&](int k) {
        g0 = make_float4(0.f, 0.f, 0.f, 0.f);
        g1 = make_float4(-1.f, 0.f, -1.f, -INFINITY);
        gc = make_float4(0.f, 0.f, 0.f, 0.f);
        gslot = kNoSlot;
        if (k >= clo) {
            const uint32_t id = a.vals[rg.x + k];
            g0 = a.geom[2 * (size_t)id];
            g1 = a.geom[2 * (size_t)id + 1];
            gc = a.color[id];
            gslot = slot_of(a, id, tx, ty);
        }
    };
    if (maxlast > clo) gather(maxlast - kBatch + lane);
    for (int hi = maxlast; hi > clo; hi -= kBatch) {
        const int lo = hi - kBatch;
        // Stage, in list order, the entries that can reach 1/255 somewhere in
        // this part's rows; a dropped entry blends nowhere there, and its slot
        // stays unwritten (flag 0, read as zero).
        const float u = rel_coord(g0.x, g0.z, px0), v = rel_coord(g0.y, g0.w, py0);
        const uint32_t mask =
            gslot != kNoSlot ? band_mask<kSplit>(u, v, g1.x, g1.y, g1.z, g1.w, row0) : 0u;
        const unsigned long long kept = __ballot(mask != 0u);
        const int nk = __popcll(kept);
        // an opacity below exp2(kLoNoClamp) keeps o exp(power) below the
        // clamp wherever power <= 0
        const bool nc_batch = __ballot(mask != 0u && !(g1.w <= kLoNoClamp)) == 0ull;
        if (mask != 0u) {
            const int r = kept_rank(kept);
            sA[r] = StagedA{u, v, g1.x, g1.y};
            sB[r] = StagedB{g1.z, g1.w, gc.x, gc.y};
            sC[r] = StagedC{gc.z, __builtin_amdgcn_exp2f(-g1.w), gslot, (uint32_t)(lo + lane)};
            sM[r] = mask;
        }
        const int nkr = (nk + kBwdUnroll - 1) & ~(kBwdUnroll - 1);
        if (lane >= nk && lane < nkr) {   // padding up to the unroll width: reaches no band
            sA[lane] = StagedA{0.f, 0.f, -1.f, 0.f};
            sB[lane] = StagedB{-1.f, -INFINITY, 0.f, 0.f};
            sC[lane] = StagedC{0.f, 0.f, kNoSlot, kPadPos};
            sM[lane] = 0u;
        }
        __syncthreads();
        if (lo > clo) gather(lo - kBatch + lane);
        // NC: no staged entry of the batch can reach the 0.99 clamp, whose
        // tests then drop out of the walk (same results, fewer operations)
        auto walk = [&](auto nc_c) __attribute__((always_inline)) {
            constexpr bool NC = decltype(nc_c)::value;
            StagedA es[kBwdUnroll];
            StagedB et[kBwdUnroll];
            StagedC ew[kBwdUnroll];
            uint32_t em[kBwdUnroll];
            auto load_group = [&](int j0, StagedA (&ra)[kBwdUnroll], StagedB (&rb)[kBwdUnroll],
                                  StagedC (&rc)[kBwdUnroll], uint32_t (&rm)[kBwdUnroll]) {
    #pragma unroll
                for (int u = 0; u < kBwdUnroll; u++) {
                    ra[u] = sA[j0 + u];
                    rb[u] = sB[j0 + u];
                    rc[u] = sC[j0 + u];
                    rm[u] = sM[j0 + u];
                }
            };
            if (GSP_BWD_PREFETCH && nkr > 0) load_group(nkr - kBwdUnroll, es, et, ew, em);
            for (int j0 = nkr - kBwdUnroll; j0 >= 0; j0 -= kBwdUnroll) {
                // the next group's records (one group ahead: the LDS round trip
                // overlaps this group's work), or this group's
                StagedA es_n[kBwdUnroll];
                StagedB et_n[kBwdUnroll];
                StagedC ew_n[kBwdUnroll];
                uint32_t em_n[kBwdUnroll];
                if (GSP_BWD_PREFETCH) {
                    load_group(j0 >= kBwdUnroll ? j0 - kBwdUnroll : 0, es_n, et_n, ew_n, em_n);
                } else {
                    load_group(j0, es, et, ew, em);
                    // All records of the group are wanted in registers here: the
                    // compiler would otherwise sink the later entries' loads
                    // below the band test, a second LDS round trip per entry.
                    // (Not in the stored-list variant, where it would cost spills.)
    #pragma unroll
                    for (int u = 0; u < (STORED ? 0 : kBwdUnroll); u++)
                        asm volatile("" ::"v"(es[u].u), "v"(es[u].v), "v"(es[u].A2), "v"(es[u].B2),
                                     "v"(et[u].C2), "v"(et[u].lo), "v"(et[u].r), "v"(et[u].g), "v"(ew[u].b),
                                     "v"(ew[u].inv_o), "v"(ew[u].slot));
                }
    #pragma unroll
                for (int u = kBwdUnroll - 1; u >= 0; u--) {
                    // the bands this entry may reach that still have pixels
                    // compositing at its list position (wave-uniform)
                    const int pos = __builtin_amdgcn_readfirstlane((int)ew[u].pm);
                    uint32_t bands = __builtin_amdgcn_readfirstlane(em[u]);
    #pragma unroll
                    for (int q = 0; q < kPixPerLane; q++)
                        if (pos >= blast[q]) bands &= ~(1u << q);
                    if (bands == 0u) continue;
                    const StagedA &s = es[u];
                    const StagedB &t = et[u];
                    const ColTerms ct = col_terms(s, fxl);
                    const float col3[3] = {t.r, t.g, ew[u].b};
                    // Per lane, dx is the same for all its pixels, so the conic
                    // and centre gradients need only the moments sum dp, sum dp dy,
                    // sum dp dy^2 of dL/dpower over them.
                    float m0 = 0.f, my = 0.f, myy = 0.f, gc[3] = {0.f, 0.f, 0.f};
                    bool blended = false;
                    // q-th pixels of all lanes form a 16 x 4 band of the tile: a
                    // band with no candidate pixel is skipped as a whole; inside a
                    // band the update is branch-free, pixels that do not blend
                    // adding exact zeros.
    #pragma unroll
                    for (int q = 0; q < kPixPerLane; q++) {
                        if (!((bands >> q) & 1u)) continue;
                        const float dy = s.v - fy[q];
                        // candidates: pixels that blend this entry, decided as
                        // the forward does (power <= 0, alpha >= 1/255), before
                        // their contributor count
                        float apre = 0.f, a0 = 0.f;
                        bool cand;
                        if (STORED) {
                            cand = npos[q] == (uint32_t)pos;
                        } else {
                            const float p2 = splat_p2(ct, t.C2, dy);
                            apre = splat_alpha_pre(p2, t.lo);
                            a0 = NC ? apre : fminf(kAlphaMax, apre);   // NC: below the clamp
                            cand = (pos < last[q]) & (p2 <= 0.f) & (a0 >= kAlphaMin);
                        }
                        if (__builtin_amdgcn_ballot_w64(cand) == 0ull) continue;
                        blended = true;
                        float alpha, wgt;
                        bool valid, unclamped;
                        if (STORED) {
                            // alpha and T_i of this pair as the forward left them
                            valid = cand;
                            alpha = valid ? fabsf(nal[q]) : 0.f;
                            unclamped = nal[q] >= 0.f;
                            wgt = valid ? alpha * T[q] : 0.f;
                        } else {
                            // A pixel that does not blend takes alpha = 0, which
                            // leaves T (times rcp(1) = 1), G.S (plus 0 * diff)
                            // and the sums (plus 0) exactly as they are.
                            valid = cand;
                            alpha = valid ? a0 : 0.f;
                            unclamped = NC || apre <= kAlphaMax;
                            T[q] = T[q] * __builtin_amdgcn_rcpf(1.f - alpha);
                            wgt = alpha * T[q];
                        }
                        const float Gc = fmaf(G[q][2], col3[2], fmaf(G[q][1], col3[1], G[q][0] * col3[0]));
                        const float diff = Gc - GS[q];
    #pragma unroll
                        for (int ch = 0; ch < 3; ch++) gc[ch] = fmaf(G[q][ch], wgt, gc[ch]);
                        GS[q] = STORED ? (valid ? fmaf(alpha, diff, GS[q]) : GS[q]) : fmaf(alpha, diff, GS[q]);
                        // dL/dpower; zero where alpha is clamped at 0.99
                        const float dp = unclamped ? wgt * diff : 0.f;
                        if (STORED && valid) {
                            // step to the pixel's previous pair (if any)
                            npos[q] = kNoPos;
                            if (pidx[q] > pbase[q]) {
                                pidx[q]--;
                                const PairRec r = a.pairs[pidx[q]];
                                npos[q] = r.pos;
                                nal[q] = r.alpha;
                                T[q] = r.T;
                            }
                        }
                        const float dpy = dp * dy;
                        m0 += dp;
                        my += dpy;
                        myy = fmaf(dpy, dy, myy);
                    }
                    if (!blended) continue;
                    {
                        // dpower/du = -(A dx + B dy), dpower/dv = -(C dy + B dx),
                        // dpower/d(A, B, C) = -(dx^2 / 2, dx dy, dy^2 / 2), in the
                        // base-2 conic and before the per-component scale below
                        float acc[9];
                        acc[0] = fmaf(s.B2, my, 2.f * s.A2 * ct.dx * m0);
                        acc[1] = fmaf(2.f * t.C2, my, ct.bdx * m0);
                        acc[2] = ct.dx * ct.dx * m0;
                        acc[3] = ct.dx * my;
                        acc[4] = myy;
                        acc[5] = OPA ? m0 : gc[0];
                        acc[6] = OPA ? gc[0] : gc[1];
                        acc[7] = OPA ? gc[1] : gc[2];
                        acc[8] = gc[2];
                        float *const dst = sP + npend * kEntryStride + (lane >> 4) * kRowStride + (lane & 15);
                        float ra, rb;
                        if (OPA) {
                            float rc;
                            wave_sum9_rows(acc, ra, rb, rc);
                            dst[2 * kRegStride] = rc;
                        } else {
                            wave_sum8_rows(acc, ra, rb);
                        }
                        dst[0] = ra;
                        dst[kRegStride] = rb;
                        if (lane == 0) {
                            sPs[npend] = ew[u].slot;
                            sPi[npend] = ew[u].inv_o;
                        }
                        if (++npend == kPend) flush();
                    }
                }
                if (GSP_BWD_PREFETCH) {
    #pragma unroll
                    for (int u = 0; u < kBwdUnroll; u++) {
                        es[u] = es_n[u];
                        et[u] = et_n[u];
                        ew[u] = ew_n[u];
                        em[u] = em_n[u];
                    }
                }
            }
        };
        if (!STORED && nc_batch) walk(std::true_type{});
        else walk(std::false_type{});
        __syncthreads();
    }
    if (npend > 0) flush();
}

hipError_t launch_raster_bwd(const ViewsK &views, const Layout &L, char *ws, const uint32_t *vals,
                             bool want_opacity, hipStream_t s) {
    if (L.total_tiles == 0) return hipSuccess;
    BwdArgs a;
    std::memset(&a, 0, sizeof a);
    a.items = region<uint32_t>(ws, L.items);
    a.counters = region<uint32_t>(ws, L.counters);
    a.ckpt = region<float4>(ws, L.ckpt);
    a.cfinal = region<float>(ws, L.cfinal);
    a.total_pix = (int)L.total_pix;
    a.ranges = region<uint2>(ws, L.ranges);
    a.vals = vals;
    a.geom = region<float4>(ws, L.geom);
    a.color = region<float4>(ws, L.color);
    a.rect = region<uint2>(ws, L.rect);
    a.offsets = region<uint32_t>(ws, L.offsets);
    a.tfinal = region<float>(ws, L.tfinal);
    a.ncontrib = region<uint32_t>(ws, L.ncontrib);
    a.slots = region<float>(ws, L.slots);
    a.slot_flags = region<uint8_t>(ws, L.slot_flags);
    // Slots that no entry writes keep the flag 0 that the forward's emission
    // stored and count as zero.  The set of written slots depends only on the
    // forward's state, so repeated backwards of one forward agree on it.
    // one workgroup per part of each possible work item; those past the
    // item count of this call exit at once
    if (want_opacity)
        hipLaunchKernelGGL((k_raster_bwd<false, true>), dim3(raster_blocks<kSplit>((int)L.max_items)),
                           dim3(kRasterThreads), 0, s, a, views);
    else
        hipLaunchKernelGGL((k_raster_bwd<false, false>), dim3(raster_blocks<kSplit>((int)L.max_items)),
                           dim3(kRasterThreads), 0, s, a, views);
    return hipGetLastError();
}

hipError_t launch_raster_bwd_stored(const ViewsK &views, const Layout &L, char *ws,
                                    const uint32_t *vals, const ListLayout &Q, const char *lists,
                                    hipStream_t s) {
    if (L.total_tiles == 0) return hipSuccess;
    BwdArgs a;
    std::memset(&a, 0, sizeof a);
    a.counters = region<uint32_t>(ws, L.counters);
    a.total_pix = (int)L.total_pix;
    a.ranges = region<uint2>(ws, L.ranges);
    a.vals = vals;
    a.geom = region<float4>(ws, L.geom);
    a.color = region<float4>(ws, L.color);
    a.rect = region<uint2>(ws, L.rect);
    a.offsets = region<uint32_t>(ws, L.offsets);
    a.slots = region<float>(ws, L.slots);
    a.slot_flags = region<uint8_t>(ws, L.slot_flags);
    a.order = region<uint32_t>(ws, L.tile_order);
    char *lw = const_cast<char *>(lists);
    a.loff = region<uint32_t>(lw, Q.offsets);
    a.pairs = region<PairRec>(lw, Q.pairs);
    a.lhdr = region<uint32_t>(lw, Q.hdr);
    a.total_tiles = L.total_tiles;
    // one workgroup per part of each tile, in the forward's launch order
    hipLaunchKernelGGL((k_raster_bwd<true, true>), dim3(raster_blocks<kSplit>(L.total_tiles)),
                       dim3(kRasterThreads), 0, s, a, views);
    return hipGetLastError();
}

}  // namespace gsp
