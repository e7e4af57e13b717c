// sort.hip -- stable LSD radix sort of (uint32 key, uint32 value) pairs.
//
// The (tile | depth) order of the instances is produced in two stable sorts
// that together equal one stable sort on the 64-bit key (tile << 32 | depth):
// the splats are first sorted by their float32 depth bits (all 32 bits, ties
// keep index order), instances are then emitted splat by splat in that order,
// and the instances are stably sorted by tile id alone (ceil(log2 tiles)
// bits).  The instance sort moves 8-byte pairs over 2 passes at a 1008x756
// view instead of 12-byte pairs over 6.
//
// Each pass is reduce-then-scan: per-block digit histograms, a per-digit
// scan across blocks, then a scatter in which every block ranks its
// kSortItems keys stably with wavefront ballots (one ballot per digit bit on
// wave64), sorts them locally in LDS and writes them out digit run by digit
// run, so global stores are contiguous within each run.  The element count
// may live in device memory (the instance count), in which case the grid is
// sized by capacity and blocks past the count exit at once: no host
// synchronisation.  The instance emission writes the first pass's
// histograms of the instance sort itself (its blocks are the sort's blocks),
// which saves that pass's histogram launch.
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
};

__device__ __forceinline__ uint32_t sort_count(const SortPass &a) {
    return a.count_ptr ? *a.count_ptr : a.count_val;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_hist(SortPass a) {
    __shared__ uint32_t h[kSortBins];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const uint32_t M = sort_count(a);
    const size_t base = (size_t)blockIdx.x * kSortItems;
    if (base < M) {
#pragma unroll 4
        for (int r = 0; r < kSortRounds; r++) {
            const size_t k = base + (size_t)r * kSortThreads + t;
            if (k < M) atomicAdd(&h[(a.keys_in[k] >> a.shift) & a.mask], 1u);
        }
    }
    __syncthreads();
    a.hist[(size_t)t * a.nblk + blockIdx.x] = h[t];
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

// With few blocks the scatter scans the histogram itself (FUSED): thread d
// sums row d of the unscanned counts over the blocks in front of its own and
// over all blocks, which saves the scan's launch.
constexpr int kFusedScanMaxBlocks = 256;

template <bool FUSED>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(SortPass a) {
    constexpr int NW = kSortThreads / kWave;
    __shared__ uint32_t skeys[kSortItems];
    __shared__ uint32_t svals[kSortItems];
    __shared__ uint32_t dstart[kSortBins];
    __shared__ uint32_t gbase[kSortBins];
    __shared__ uint32_t run[kSortBins];
    __shared__ uint32_t wcnt[NW][kSortBins];
    __shared__ uint32_t wpre[NW][kSortBins];
    __shared__ uint32_t scratch[kSortThreads / kWave];

    const uint32_t M = sort_count(a);
    const size_t base = (size_t)blockIdx.x * kSortItems;
    if (base >= M) return;
    const int cnt = (int)min((size_t)kSortItems, (size_t)M - base);
    const int t = threadIdx.x;
    const int lane = t & (kWave - 1);
    const int w = t / kWave;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;

    uint32_t key[kSortRounds], val[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; r++) {
        const int k = r * kSortThreads + t;
        key[r] = k < cnt ? a.keys_in[base + k] : 0u;
        val[r] = k < cnt ? a.vals_in[base + k] : 0u;
    }

    // local histogram -> local digit starts
    run[t] = 0;
#pragma unroll
    for (int w2 = 0; w2 < NW; w2++) wcnt[w2][t] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; r++) {
        if (r * kSortThreads + t < cnt) atomicAdd(&run[(key[r] >> a.shift) & a.mask], 1u);
    }
    __syncthreads();
    uint32_t tot;
    const uint32_t excl = block_exclusive_scan<uint32_t, kSortThreads>(run[t], scratch, &tot);
    uint32_t digit_total, before;
    if (FUSED) {
        const uint32_t *row = a.hist + (size_t)t * a.nblk;
        uint32_t s0 = 0, s1 = 0, b0 = 0, b1 = 0;
        const int me = (int)blockIdx.x;
        int k = 0;
        for (; k + 1 < a.nblk; k += 2) {
            const uint32_t x0 = row[k], x1 = row[k + 1];
            s0 += x0;
            s1 += x1;
            b0 += k < me ? x0 : 0u;
            b1 += k + 1 < me ? x1 : 0u;
        }
        if (k < a.nblk) {
            s0 += row[k];
            b0 += k < me ? row[k] : 0u;
        }
        digit_total = s0 + s1;
        before = b0 + b1;
    } else {
        digit_total = a.digit_tot[t];
        before = a.hist[(size_t)t * a.nblk + blockIdx.x];
    }
    const uint32_t dex = block_exclusive_scan<uint32_t, kSortThreads>(digit_total, scratch, &tot);
    dstart[t] = excl;
    run[t] = excl;
    gbase[t] = dex + before;
    __syncthreads();

    // stable ranking, round by round, wave by wave, lane by lane
#pragma unroll 1
    for (int r = 0; r < kSortRounds; r++) {
        const bool valid = r * kSortThreads + t < cnt;
        const uint32_t d = (key[r] >> a.shift) & a.mask;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kSortBits; b++) {
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
            svals[pos] = val[r];
        }
    }
    __syncthreads();

    for (int i = t; i < cnt; i += kSortThreads) {
        const uint32_t k = skeys[i];
        const uint32_t d = (k >> a.shift) & a.mask;
        const size_t dst = (size_t)gbase[d] + (uint32_t)(i - dstart[d]);
        a.keys_out[dst] = k;
        a.vals_out[dst] = svals[i];
    }
}

int launch_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, uint32_t *hist,
                      uint32_t *digit_tot, const uint32_t *count_ptr, uint32_t count_val,
                      int64_t max_count, int bits, bool hist0_given, hipStream_t s,
                      hipError_t *err) {
    SortPass a;
    a.hist = hist;
    a.digit_tot = digit_tot;
    a.count_ptr = count_ptr;
    a.count_val = count_val;
    a.nblk = (int)((max_count + kSortItems - 1) / kSortItems);
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
        a.shift = p * pbits;
        if (p > 0 || !hist0_given)
            hipLaunchKernelGGL(k_sort_hist, dim3(a.nblk), dim3(kSortThreads), 0, s, a);
        if (a.nblk <= kFusedScanMaxBlocks) {
            hipLaunchKernelGGL(k_sort_scatter<true>, dim3(a.nblk), dim3(kSortThreads), 0, s, a);
        } else {
            hipLaunchKernelGGL(k_sort_scan, dim3(kSortBins), dim3(kSortScanThreads), 0, s, a);
            hipLaunchKernelGGL(k_sort_scatter<false>, dim3(a.nblk), dim3(kSortThreads), 0, s, a);
        }
        *err = hipGetLastError();
        if (*err != hipSuccess) return passes;
    }
    return passes;
}

hipError_t launch_depth_sort(const Layout &L, char *ws, hipStream_t s) {
    hipError_t e;
    launch_sort_pairs(region<uint32_t>(ws, L.dkeys0), region<uint32_t>(ws, L.dvals0),
                      region<uint32_t>(ws, L.dkeys1), region<uint32_t>(ws, L.dvals1),
                      region<uint32_t>(ws, L.hist), region<uint32_t>(ws, L.digit_tot), nullptr,
                      (uint32_t)L.vn, L.vn, 32, false, s, &e);
    return e;
}

hipError_t launch_tile_sort(const Layout &L, char *ws, hipStream_t s) {
    hipError_t e;
    launch_sort_pairs(region<uint32_t>(ws, L.keys0), region<uint32_t>(ws, L.vals0),
                      region<uint32_t>(ws, L.keys1), region<uint32_t>(ws, L.vals1),
                      region<uint32_t>(ws, L.hist), region<uint32_t>(ws, L.digit_tot),
                      region<uint32_t>(ws, L.counters) + kCntMEff, 0u, L.cap, L.tile_bits, true, s,
                      &e);
    return e;
}

}  // namespace gsp
