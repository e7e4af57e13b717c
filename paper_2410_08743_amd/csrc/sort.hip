// sort.hip -- the (tile, depth, index) order of the instances.
//
// The order of one stable sort on the 64-bit key (tile << 32 | depth) is
// produced in two steps: the instances, emitted splat by splat in index
// order, are stably sorted by tile id alone (ceil(log2 tiles) bits, 2 passes
// at a 1008x756 view; 8-byte pairs), and then each tile's run, now in index
// order, is sorted stably by depth inside one workgroup (k_tile_depth_sort,
// at the end of this file).  Sorting the depth per tile in LDS replaces a
// global depth sort of all splats (4 passes of 3 launches each).
//
// Each pass is reduce-then-scan: per-block digit histograms, a per-digit
// scan across blocks, then a scatter in which every block ranks its
// 1024 or 2048 keys stably with wavefront ballots (one ballot per digit bit on
// wave64), sorts them locally in LDS and writes them out digit run by digit
// run, so global stores are contiguous within each run.  The element count
// may live in device memory (the instance count), in which case the grid is
// sized by capacity and blocks past the count exit at once: no host
// synchronisation.  The instance emission writes the first pass's
// histograms of the instance sort itself (its blocks are the sort's blocks),
// which saves that pass's histogram launch.
#include <type_traits>

#include "block_ops.h"
#include "gsp_internal.h"

namespace gsp {

struct SortPass {
    const uint32_t *keys_in;
    const uint32_t *vals_in;
    uint32_t *keys_out;
    uint32_t *vals_out;
    uint32_t *hist;        // [bins][nblk]
    uint32_t *digit_tot;   // [bins]
    const uint32_t *count_ptr;  // element count in device memory, or null
    uint32_t count_val;         // element count when count_ptr is null
    int nblk;
    int shift;
    uint32_t mask;     // digit mask of this pass (at most kSortBins - 1)
    int vbits;         // packed items: the value's bits below the key
};

// Item layout of a pass: a key and a value array (kPairs); one word per
// item, the key above the value's vbits bits (kPacked, when the tile bits
// and the value bits fit 32 between them); or packed items in and the two
// arrays out (kUnpack, the last pass of a packed sort).
enum SortMode { kPairs = 0, kPacked = 1, kUnpack = 2 };

__device__ __forceinline__ uint32_t sort_count(const SortPass &a) {
    return a.count_ptr ? *a.count_ptr : a.count_val;
}

template <int R>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(SortPass a) {
    constexpr int kItems = kSortThreads * R;
    __shared__ uint32_t h[kSortBins];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const uint32_t M = sort_count(a);
    const size_t base = (size_t)blockIdx.x * kItems;
    if (base < M) {
#pragma unroll 4
        for (int r = 0; r < R; r++) {
            const size_t k = base + (size_t)r * kSortThreads + t;
            if (k < M) atomicAdd(&h[(a.keys_in[k] >> a.shift) & a.mask], 1u);
        }
    }
    __syncthreads();
    if ((uint32_t)t <= a.mask) a.hist[(size_t)t * a.nblk + blockIdx.x] = h[t];   // rows of used digits
}

// One block per digit: exclusive scan of that digit's counts across blocks
// (a row of up to tens of thousands of counts for the instance sort of a
// multi-view call).  The row is scanned in chunks of 4 x 1024 counts: each
// thread loads four consecutive counts of the chunk (the wave's loads cover
// 1 KB contiguously), the block scans the per-thread sums, and the running
// total carries from chunk to chunk.
constexpr int kSortScanThreads = 1024;
constexpr int kSortScanChunk = 4 * kSortScanThreads;

__global__ __launch_bounds__(kSortScanThreads) void k_sort_scan(SortPass a) {
    __shared__ uint32_t scratch[kSortScanThreads / kWave];
    const int t = threadIdx.x;
    uint32_t *row = a.hist + (size_t)blockIdx.x * a.nblk;
    uint32_t carry = 0;
    for (int c0 = 0; c0 < a.nblk; c0 += kSortScanChunk) {
        const int k0 = c0 + 4 * t;
        uint32_t x[4];
#pragma unroll
        for (int j = 0; j < 4; j++) x[j] = k0 + j < a.nblk ? row[k0 + j] : 0u;
        const uint32_t local = x[0] + x[1] + x[2] + x[3];
        uint32_t total;
        uint32_t off = carry + block_exclusive_scan<uint32_t, kSortScanThreads>(local, scratch, &total);
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (k0 + j < a.nblk) row[k0 + j] = off;
            off += x[j];
        }
        carry += total;
    }
    if (t == 0) a.digit_tot[blockIdx.x] = carry;
}

template <int R, int MODE>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(SortPass a) {
    constexpr int NW = kSortThreads / kWave;
    constexpr int kItems = kSortThreads * R;
    __shared__ uint32_t skeys[kItems];
    __shared__ uint32_t svals[MODE == kPairs ? kItems : 1];
    __shared__ uint32_t dstart[kSortBins];
    __shared__ uint32_t gbase[kSortBins];
    __shared__ uint32_t run[kSortBins];
    __shared__ uint32_t wcnt[NW][kSortBins];
    __shared__ uint32_t wpre[NW][kSortBins];
    __shared__ uint32_t scratch[kSortThreads / kWave];

    const uint32_t M = sort_count(a);
    const size_t base = (size_t)blockIdx.x * kItems;
    if (base >= M) return;
    const int cnt = (int)min((size_t)kItems, (size_t)M - base);
    const int t = threadIdx.x;
    const int lane = t & (kWave - 1);
    const int w = t / kWave;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;

    uint32_t key[R], val[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int k = r * kSortThreads + t;
        key[r] = k < cnt ? a.keys_in[base + k] : 0u;
        val[r] = MODE == kPairs && k < cnt ? a.vals_in[base + k] : 0u;
    }

    // local histogram -> local digit starts
    run[t] = 0;
#pragma unroll
    for (int w2 = 0; w2 < NW; w2++) wcnt[w2][t] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; r++) {
        if (r * kSortThreads + t < cnt) atomicAdd(&run[(key[r] >> a.shift) & a.mask], 1u);
    }
    __syncthreads();
    uint32_t tot;
    const uint32_t excl = block_exclusive_scan<uint32_t, kSortThreads>(run[t], scratch, &tot);
    // rows and totals exist for the pass's digits only (mask + 1 of them)
    const bool used = (uint32_t)t <= a.mask;
    const uint32_t digit_total = used ? a.digit_tot[t] : 0u;
    const uint32_t before = used ? a.hist[(size_t)t * a.nblk + blockIdx.x] : 0u;
    const uint32_t dex = block_exclusive_scan<uint32_t, kSortThreads>(digit_total, scratch, &tot);
    dstart[t] = excl;
    run[t] = excl;
    gbase[t] = dex + before;
    __syncthreads();

    // stable ranking, round by round, wave by wave, lane by lane
#pragma unroll 1
    for (int r = 0; r < R; r++) {
        const bool valid = r * kSortThreads + t < cnt;
        const uint32_t d = (key[r] >> a.shift) & a.mask;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kSortBits; b++) {
            if (!((a.mask >> b) & 1u)) break;   // the pass's digit bits only
            const bool bit = (d >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        if (!valid) peers = 0;
        const uint32_t rank = __popcll(peers & lt_mask);
        if (valid && (peers & lt_mask) == 0) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        {
            uint32_t acc = run[t];
#pragma unroll
            for (int w2 = 0; w2 < NW; w2++) {
                const uint32_t c = wcnt[w2][t];
                wcnt[w2][t] = 0;
                wpre[w2][t] = acc;
                acc += c;
            }
            run[t] = acc;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wpre[w][d] + rank;
            skeys[pos] = key[r];
            if (MODE == kPairs) svals[pos] = val[r];
        }
    }
    __syncthreads();

    for (int i = t; i < cnt; i += kSortThreads) {
        const uint32_t k = skeys[i];
        const uint32_t d = (k >> a.shift) & a.mask;
        const size_t dst = (size_t)gbase[d] + (uint32_t)(i - dstart[d]);
        if (MODE == kPairs) {
            a.keys_out[dst] = k;
            a.vals_out[dst] = svals[i];
        } else if (MODE == kPacked) {
            a.keys_out[dst] = k;
        } else {
            a.keys_out[dst] = k >> a.vbits;
            a.vals_out[dst] = k & ((1u << a.vbits) - 1u);
        }
    }
}

// vbits > 0: the input is packed (k0 only) and the passes before the last
// keep it packed; the last pass writes keys and values.
template <int R>
static int launch_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, uint32_t *hist,
                             uint32_t *digit_tot, const uint32_t *count_ptr, uint32_t count_val,
                             int64_t max_count, int bits, bool hist0_given, int vbits, hipStream_t s,
                             hipError_t *err) {
    constexpr int kItems = kSortThreads * R;
    SortPass a;
    a.hist = hist;
    a.digit_tot = digit_tot;
    a.count_ptr = count_ptr;
    a.count_val = count_val;
    a.nblk = (int)((max_count + kItems - 1) / kItems);
    *err = hipSuccess;
    const int passes = sort_passes(bits);
    const int pbits = digit_bits(bits);
    a.mask = (1u << pbits) - 1u;
    if (a.nblk == 0) return passes;
    for (int p = 0; p < passes; p++) {
        a.keys_in = (p & 1) ? k1 : k0;
        a.vals_in = (p & 1) ? v1 : v0;
        a.keys_out = (p & 1) ? k0 : k1;
        a.vals_out = (p & 1) ? v0 : v1;
        a.shift = vbits + p * pbits;
        a.vbits = vbits;
        if (p > 0 || !hist0_given)
            hipLaunchKernelGGL(k_sort_hist<R>, dim3(a.nblk), dim3(kSortThreads), 0, s, a);
        hipLaunchKernelGGL(k_sort_scan, dim3(a.mask + 1), dim3(kSortScanThreads), 0, s, a);
        if (vbits == 0)
            hipLaunchKernelGGL((k_sort_scatter<R, kPairs>), dim3(a.nblk), dim3(kSortThreads), 0, s, a);
        else if (p < passes - 1)
            hipLaunchKernelGGL((k_sort_scatter<R, kPacked>), dim3(a.nblk), dim3(kSortThreads), 0, s, a);
        else
            hipLaunchKernelGGL((k_sort_scatter<R, kUnpack>), dim3(a.nblk), dim3(kSortThreads), 0, s, a);
        *err = hipGetLastError();
        if (*err != hipSuccess) return passes;
    }
    return passes;
}

hipError_t launch_tile_sort(const Layout &L, char *ws, hipStream_t s) {
    hipError_t e;
    auto run = [&](auto rounds) {
        launch_sort_pairs<decltype(rounds)::value>(
            region<uint32_t>(ws, L.keys0), region<uint32_t>(ws, L.vals0), region<uint32_t>(ws, L.keys1),
            region<uint32_t>(ws, L.vals1), region<uint32_t>(ws, L.hist), region<uint32_t>(ws, L.digit_tot),
            region<uint32_t>(ws, L.counters) + kCntMEff, 0u, L.cap, L.tile_bits, true, L.sort_vbits, s,
            &e);
    };
    if (L.sort_items == kSortThreads * kSortRoundsLarge)
        run(std::integral_constant<int, kSortRoundsLarge>{});
    else
        run(std::integral_constant<int, kSortRoundsSmall>{});
    return e;
}


// ---------------------------------------------------------------------------
// Depth order inside each tile.  The instances leave the tile sort grouped by
// tile, each tile's run in index order (they are emitted splat by splat in
// index order and the tile sort is stable).  Each tile's run is then sorted
// stably by the splat's depth key (the float32 bits of its camera-frame z):
// equal depths keep index order, so every run ends in (depth, index) order,
// which is the order of a stable sort of all instances on the 64-bit key
// (tile << 32 | depth).  Only the values (view * n + i) move.
//
// One wavefront per tile (a 64-thread workgroup, so that its barriers cost
// nothing and many tiles are in flight per CU); workgroup b takes tile b, so
// that its first load is its range.  The keys are taken relative to the
// run's smallest (an order-preserving shift that leaves some 25 significant
// bits for depths in 1.5 .. 8) and sorted LSD over kTdBits-bit digits (9:
// three passes over those 25 bits, where 8-bit digits take four),
// skipping every pass whose digit is the same for the whole run.  A pass is a
// stable counting sort: rounds of 64 items, each lane ranked among the
// round's lanes with the same digit (found through a per-digit lane mask in
// LDS) on top of a running per-digit count, then the digit counts' exclusive
// scan added to those ranks.  Runs of up to CAP entries stay in registers
// and LDS (CAP is picked per launch from the mean list length the instance
// capacity allows: 1024 or 2048), one 32-bit word per item: after the first
// pass the relative key's remaining bits sit above the item's position in
// the run, and the values are gathered by that position once at the end (so
// a pass scatters and reloads one word per item, and LDS holds CAP words).
// Longer runs, and runs whose keys are too wide for that packing (depths
// spread over some sixty binary orders of magnitude), sorted over 8-bit
// digits (histograms of every pass from one read first), move, CAP entries at a time with every load of a chunk in
// flight, between the sorted arrays and the tile sort's other key and value
// buffers, the relative keys carried beside the values (the key array's
// tile ids are restored afterwards).
#ifndef GSP_TD_BITS
#define GSP_TD_BITS 9
#endif
// digits of the runs sorted in LDS (three passes over 25 significant bits)
constexpr int kTdBits = GSP_TD_BITS;
constexpr int kTdBins = 1 << kTdBits;
// digits of the long runs, whose histograms of all passes share buf
constexpr int kTdLBits = 8;
constexpr int kTdLBins = 1 << kTdLBits;
constexpr int kTdLPasses = (32 + kTdLBits - 1) / kTdLBits;
static_assert(kTdBits >= kTdLBits && kTdBins % kWave == 0, "run and msk hold either digit");

struct TileDepthArgs {
    const uint2 *ranges;
    const uint32_t *depth;      // [vn] depth key of each view-Gaussian
    uint32_t *keys;             // sorted tile ids (scratch for long runs, then restored)
    uint32_t *vals;             // sorted values, put in depth order per tile in place
    uint32_t *akeys, *avals;    // [cap] the tile sort's other buffers (scratch)
};

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, off, kWave));
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, kWave));
    return v;
}

// Rank of the lane's item among the lanes of its round with the same digit,
// plus run[d], the count of d in earlier rounds.  The lanes with digit d find
// each other through msk[d]: each ORs its lane bit in, then reads the mask
// back (a wavefront's LDS accesses take effect in program order, so every OR
// lands before any read); the lowest of them advances run[d] and clears
// msk[d] for the next round.  msk must be zero on entry and is zero again on
// return.
__device__ __forceinline__ uint32_t td_rank(bool valid, uint32_t d, uint32_t *run,
                                            unsigned long long *msk) {
    const int lane = threadIdx.x;
    const unsigned long long lt = (1ull << lane) - 1ull;
    if (valid) atomicOr(&msk[d], 1ull << lane);
    const unsigned long long peers = valid ? msk[d] : 0ull;
    const uint32_t below = __popcll(peers & lt);
    const uint32_t base = valid ? run[d] : 0u;
    if (valid && below == 0) {
        run[d] = base + (uint32_t)__popcll(peers);
        msk[d] = 0ull;
    }
    return base + below;
}

// run[] (digit counts of BINS digits) -> exclusive starts, in place.
template <int BINS>
__device__ __forceinline__ void td_scan(uint32_t *run) {
    constexpr int kTdPerLane = BINS / kWave;
    const int lane = threadIdx.x;
    uint32_t c[kTdPerLane], s = 0;
#pragma unroll
    for (int j = 0; j < kTdPerLane; j++) {
        c[j] = run[kTdPerLane * lane + j];
        s += c[j];
    }
    uint32_t e = wave_inclusive_scan(s) - s;
#pragma unroll
    for (int j = 0; j < kTdPerLane; j++) {
        run[kTdPerLane * lane + j] = e;
        e += c[j];
    }
    __syncthreads();
}

template <int BINS>
__device__ __forceinline__ void td_zero(uint32_t *run) {
    constexpr int kTdPerLane = BINS / kWave;
#pragma unroll
    for (int j = 0; j < kTdPerLane; j++) run[kTdPerLane * threadIdx.x + j] = 0u;
}

// An overflowing forward emits no instance and leaves every range empty, so
// the kernel needs no overflow test.
template <int CAP>
__global__ __launch_bounds__(kWave) void k_tile_depth_sort(TileDepthArgs a) {
    constexpr int kTdCap = CAP;
    constexpr int kTdRounds = kTdCap / kWave;
    constexpr int kIdx = CAP == 2048 ? 11 : 10;   // bits of a position in the run
    static_assert((1 << kIdx) == kTdCap, "CAP is 1024 or 2048");
    // the run's packed items (long runs: the histograms of all passes instead)
    __shared__ uint32_t buf[kTdCap];
    __shared__ uint32_t run[kTdBins];
    __shared__ unsigned long long msk[kTdBins];
    static_assert(kTdLPasses * kTdLBins <= kTdCap, "histograms of a long run fit in buf");
    const uint32_t tile = blockIdx.x;
    const uint2 rg = a.ranges[tile];
    const int L = (int)(rg.y - rg.x);
    if (L <= 1) return;
    const int lane = threadIdx.x;
    uint32_t key[kTdRounds], val[kTdRounds];
    uint32_t *const kf = a.keys + rg.x, *const vf = a.vals + rg.x;
#pragma unroll
    for (int j = 0; j < kTdBins / kWave; j++) msk[kTdBins / kWave * lane + j] = 0ull;

    if (L <= kTdCap) {
#pragma unroll
        for (int r = 0; r < kTdRounds; r++) {
            const int k = r * kWave + lane;
            val[r] = k < L ? vf[k] : 0u;
        }
        uint32_t kmin = 0xffffffffu, kmax = 0u;
#pragma unroll
        for (int r = 0; r < kTdRounds; r++) {
            const int k = r * kWave + lane;
            key[r] = k < L ? a.depth[val[r]] : 0u;
            if (k < L) {
                kmin = min(kmin, key[r]);
                kmax = max(kmax, key[r]);
            }
        }
        kmin = wave_min_u32(kmin);
        kmax = wave_max_u32(kmax);
        // significant bits of the relative keys; runs whose keys span more
        // than 32 - kIdx + 8 bits (depths over some sixty binary orders of
        // magnitude) take the long path below
        const int B = kmax > kmin ? 32 - __clz(kmax - kmin) : 0;
        if (B <= 32 - kIdx + kTdBits) {
            // An item is one word: after the first pass, the relative key's
            // bits above that pass's digit, shifted over the item's position
            // in the run (kIdx bits); the values follow by that position at
            // the end.  One LDS word per item and pass, not two.
            uint32_t pk[kTdRounds], rk[kTdRounds];
            bool moved = false;
            // One counting-sort pass over digit d(r) of the items pk (the
            // first pass's items and digits come from the relative keys).
            auto sort_pass = [&](auto digit_of, auto item_of) {
                uint32_t dlo = kTdBins, dhi = 0;
#pragma unroll
                for (int r = 0; r < kTdRounds; r++) {
                    if (r * kWave + lane < L) {
                        const uint32_t d = digit_of(r);
                        dlo = min(dlo, d);
                        dhi = max(dhi, d);
                    }
                }
                if (wave_min_u32(dlo) == wave_max_u32(dhi)) {   // one digit: nothing moves
#pragma unroll
                    for (int r = 0; r < kTdRounds; r++) pk[r] = item_of(r);
                    return;
                }
                moved = true;
                td_zero<kTdBins>(run);
                __syncthreads();
#pragma unroll
                for (int r = 0; r < kTdRounds; r++) {
                    rk[r] = 0u;
                    if (r * kWave >= L) continue;   // uniform
                    const bool valid = r * kWave + lane < L;
                    rk[r] = td_rank(valid, digit_of(r), run, msk);
                }
                __syncthreads();
                td_scan<kTdBins>(run);
#pragma unroll
                for (int r = 0; r < kTdRounds; r++)
                    if (r * kWave + lane < L) buf[run[digit_of(r)] + rk[r]] = item_of(r);
                __syncthreads();
#pragma unroll
                for (int r = 0; r < kTdRounds; r++) {
                    const int k = r * kWave + lane;
                    pk[r] = k < L ? buf[k] : 0u;
                }
                __syncthreads();
            };
            // pass 0: the relative keys' low digit; items become (key bits
            // above it, position)
#pragma unroll
            for (int r = 0; r < kTdRounds; r++) key[r] -= kmin;
            sort_pass([&](int r) { return key[r] & (kTdBins - 1); },
                      [&](int r) { return ((key[r] >> kTdBits) << kIdx) | (uint32_t)(r * kWave + lane); });
            const int npass = (B + kTdBits - 1) / kTdBits;
            for (int p = 1; p < npass; p++) {
                const int sh = kIdx + kTdBits * (p - 1);
                sort_pass([&](int r) { return (pk[r] >> sh) & (kTdBins - 1); }, [&](int r) { return pk[r]; });
            }
            if (moved) {
                // every value read (by its position in the run) before any is written
#pragma unroll
                for (int r = 0; r < kTdRounds; r++) {
                    const int k = r * kWave + lane;
                    val[r] = k < L ? vf[pk[r] & (kTdCap - 1)] : 0u;
                }
#pragma unroll
                for (int r = 0; r < kTdRounds; r++) {
                    const int k = r * kWave + lane;
                    if (k < L) vf[k] = val[r];
                }
            }
            return;
        }
    }

    // Long run.  The smallest key, then the histograms of every pass of the
    // relative keys, from two reads of the run (keys gathered).
    uint32_t kmin = 0xffffffffu;
    for (int c0 = 0; c0 < L; c0 += kTdCap) {
#pragma unroll
        for (int r = 0; r < kTdRounds; r++) {
            const int k = c0 + r * kWave + lane;
            val[r] = k < L ? vf[k] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kTdRounds; r++) {
            const int k = c0 + r * kWave + lane;
            if (k < L) kmin = min(kmin, a.depth[val[r]]);
        }
    }
    kmin = wave_min_u32(kmin);
    uint32_t *const hist = buf;   // [kTdLPasses][kTdLBins]
    for (int i = lane; i < kTdLPasses * kTdLBins; i += kWave) hist[i] = 0u;
    __syncthreads();
    for (int c0 = 0; c0 < L; c0 += kTdCap) {
#pragma unroll
        for (int r = 0; r < kTdRounds; r++) {
            const int k = c0 + r * kWave + lane;
            val[r] = k < L ? vf[k] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kTdRounds; r++) {
            const int k = c0 + r * kWave + lane;
            if (k < L) {
                const uint32_t kk = a.depth[val[r]] - kmin;
#pragma unroll
                for (int p = 0; p < kTdLPasses; p++)
                    atomicAdd(&hist[p * kTdLBins + ((kk >> (kTdLBits * p)) & (kTdLBins - 1))], 1u);
            }
        }
    }
    __syncthreads();
    // source of the next pass: (keys gathered | skey, sval), destination (dkey, dval)
    uint32_t *skey = nullptr, *sval = vf, *dkey = a.akeys + rg.x, *dval = a.avals + rg.x;
    bool kf_used = false;
    for (int p = 0; p < kTdLPasses; p++) {
        const int sh = kTdLBits * p;
        constexpr int kTdPerLane = kTdLBins / kWave;
        bool full = false;
#pragma unroll
        for (int j = 0; j < kTdPerLane; j++) {
            const uint32_t c = hist[p * kTdLBins + kTdPerLane * lane + j];
            full |= c == (uint32_t)L;
            run[kTdPerLane * lane + j] = c;
        }
        if (wave_any(full)) continue;   // one digit: nothing moves
        __syncthreads();
        td_scan<kTdLBins>(run);
        for (int c0 = 0; c0 < L; c0 += kTdCap) {
#pragma unroll
            for (int r = 0; r < kTdRounds; r++) {
                const int k = c0 + r * kWave + lane;
                val[r] = k < L ? sval[k] : 0u;
                key[r] = k < L && skey ? skey[k] : 0u;
            }
            if (!skey) {
#pragma unroll
                for (int r = 0; r < kTdRounds; r++) {
                    const int k = c0 + r * kWave + lane;
                    key[r] = k < L ? a.depth[val[r]] - kmin : 0u;
                }
            }
#pragma unroll
            for (int r = 0; r < kTdRounds; r++) {
                if (c0 + r * kWave >= L) break;   // uniform
                const bool valid = c0 + r * kWave + lane < L;
                const uint32_t pos = td_rank(valid, (key[r] >> sh) & (kTdLBins - 1), run, msk);
                if (valid) {
                    dkey[pos] = key[r];
                    dval[pos] = val[r];
                }
            }
        }
        // the next pass reads what every lane wrote
        __syncthreads();
        kf_used |= dkey == kf;
        uint32_t *const nk = dkey == kf ? a.akeys + rg.x : kf;
        uint32_t *const nv = dval == vf ? a.avals + rg.x : vf;
        skey = dkey;
        sval = dval;
        dkey = nk;
        dval = nv;
    }
    if (sval != vf) {
        for (int c0 = 0; c0 < L; c0 += kTdCap) {
#pragma unroll
            for (int r = 0; r < kTdRounds; r++) {
                const int k = c0 + r * kWave + lane;
                val[r] = k < L ? sval[k] : 0u;
            }
#pragma unroll
            for (int r = 0; r < kTdRounds; r++) {
                const int k = c0 + r * kWave + lane;
                if (k < L) vf[k] = val[r];
            }
        }
    }
    if (kf_used)
        for (int k = lane; k < L; k += kWave) kf[k] = tile;
}

hipError_t launch_tile_depth_sort(const Layout &L, char *ws, hipStream_t s) {
    if (L.total_tiles == 0) return hipSuccess;
    TileDepthArgs a;
    const bool odd = sorted_vals(L) == L.vals1;
    a.ranges = region<uint2>(ws, L.ranges);
    a.depth = region<uint32_t>(ws, L.depth);
    a.keys = region<uint32_t>(ws, sorted_keys(L));
    a.vals = region<uint32_t>(ws, sorted_vals(L));
    a.akeys = region<uint32_t>(ws, odd ? L.keys0 : L.keys1);
    a.avals = region<uint32_t>(ws, odd ? L.vals0 : L.vals1);
    // lists longer than 1024 on average (at the 1.5x capacity margin) take the
    // 2048-entry variant, whose larger LDS share lowers the waves per CU
    if (L.cap > (int64_t)1536 * L.total_tiles)
        hipLaunchKernelGGL(k_tile_depth_sort<2048>, dim3(L.total_tiles), dim3(kWave), 0, s, a);
    else
        hipLaunchKernelGGL(k_tile_depth_sort<1024>, dim3(L.total_tiles), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

}  // namespace gsp
